// gf_sweep_sr.hip -- stochastic-relaxation half-sweeps (gf_sweep_sr).
#include "gf_host.hpp"

gf_status gf_sweep_sr(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, int32_t parity,
                      double omega, double prob, uint64_t seed, uint64_t sweep) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_sweep_sr");
  CHECK_GAUGE_PARITY(c, gauge, parity, "gf_sweep_sr");
  REJECT_MAG(c, gauge, "gf_sweep_sr");
  if (!U) return fail(c, GF_ERR_ARG, "gf_sweep_sr: NULL field");
  if (!(omega >= 1.0 && omega < 2.0)) return fail(c, GF_ERR_ARG, "gf_sweep_sr: omega must be in [1, 2)");
  if (!(prob >= 0.0 && prob <= 1.0)) return fail(c, GF_ERR_ARG, "gf_sweep_sr: prob must be in [0, 1]");
  return launch_update(
      c, U, g, gauge, parity,
      [&]<typename T>() {
        UpdSR<T> u;
        u.omega = (T)omega;
        u.prob = prob;
        u.k0 = (uint32_t)seed;
        u.k1 = (uint32_t)(seed >> 32);
        u.sweep = (uint32_t)sweep;
        return u;
      },
      "gf_sweep_sr");
}
