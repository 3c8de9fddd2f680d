// gf_anneal.hip -- annealing half-sweeps: heatbath and microcanonical.
#include "gf_host.hpp"

gf_status gf_micro_half(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, int32_t parity) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_micro_half");
  CHECK_GAUGE_PARITY(c, gauge, parity, "gf_micro_half");
  REJECT_MAG(c, gauge, "gf_micro_half");
  if (!U) return fail(c, GF_ERR_ARG, "gf_micro_half: NULL field");
  return launch_update(
      c, U, g, gauge, parity, [&]<typename T>() { return UpdMicro<T>(); }, "gf_micro_half");
}

gf_status gf_heatbath_half(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, int32_t parity,
                           double T, uint64_t seed, uint64_t sweep) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_heatbath_half");
  CHECK_GAUGE_PARITY(c, gauge, parity, "gf_heatbath_half");
  REJECT_MAG(c, gauge, "gf_heatbath_half");
  if (!U) return fail(c, GF_ERR_ARG, "gf_heatbath_half: NULL field");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(c, GF_ERR_ARG, "gf_heatbath_half: T must be > 0");
  return launch_update(
      c, U, g, gauge, parity,
      [&]<typename TT>() {
        UpdHB<TT> u;
        u.temp = (TT)T;
        u.k0 = (uint32_t)seed;
        u.k1 = (uint32_t)(seed >> 32);
        u.sweep = (uint32_t)sweep;
        return u;
      },
      "gf_heatbath_half");
}

gf_status gf_anneal_sweep(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, double T,
                          uint64_t seed, uint64_t sweep, int32_t n_micro) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_anneal_sweep");
  REJECT_MAG(c, gauge, "gf_anneal_sweep");
  if (gauge != GF_LANDAU && gauge != GF_COULOMB) return fail(c, GF_ERR_ARG, "gf_anneal_sweep: bad gauge");
  if (!U) return fail(c, GF_ERR_ARG, "gf_anneal_sweep: NULL field");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(c, GF_ERR_ARG, "gf_anneal_sweep: T must be > 0");
  if (n_micro < 0) return fail(c, GF_ERR_ARG, "gf_anneal_sweep: n_micro < 0");
  gf_status st;
  for (int p = 0; p < 2; ++p)
    if ((st = gf_heatbath_half(c, U, g, gauge, p, T, seed, sweep)) != GF_OK) return st;
  for (int k = 0; k < n_micro; ++k)
    for (int p = 0; p < 2; ++p)
      if ((st = gf_micro_half(c, U, g, gauge, p)) != GF_OK) return st;
  return GF_OK;
}
