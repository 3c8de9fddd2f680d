// gf_sweep_or.hip -- the overrelaxation half-sweep (gf_sweep).
#include "gf_host.hpp"

gf_status gf_sweep(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, int32_t parity,
                   double omega) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_sweep");
  CHECK_GAUGE_PARITY(c, gauge, parity, "gf_sweep");
  if (!U) return fail(c, GF_ERR_ARG, "gf_sweep: NULL field");
  if (!(omega >= 1.0 && omega < 2.0)) return fail(c, GF_ERR_ARG, "gf_sweep: omega must be in [1, 2)");
  return launch_update(
      c, U, g, gauge, parity,
      [&]<typename T>() {
        UpdOR<T> u;
        u.omega = (T)omega;
        return u;
      },
      "gf_sweep");
}
