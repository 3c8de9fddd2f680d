// gf_tracked_anneal.hip -- FP32 stochastic-relaxation and annealing
// half-sweeps with the site transformations accumulated into a
// gauge-transformation field.
#include "gf_host.hpp"

gf_status sweep_sr_tracked(gf_ctx* c, void* U, void* Gx, const gf_geom* g, int32_t gauge,
                                  int32_t parity, double omega, double prob, uint64_t seed,
                                  uint64_t sweep) {
  UpdSR<float> upd;
  upd.omega = (float)omega;
  upd.prob = prob;
  upd.k0 = (uint32_t)seed;
  upd.k1 = (uint32_t)(seed >> 32);
  upd.sweep = (uint32_t)sweep;
  return update_tracked(c, U, Gx, g, gauge, parity, upd, "tracked stochastic relaxation");
}

// one annealing step on an FP32 field with g tracking
gf_status anneal_step_tracked(gf_ctx* c, void* U, void* Gx, const gf_geom* g, int32_t gauge,
                                     double T, uint64_t seed, uint64_t sweep, int32_t n_micro) {
  UpdHB<float> hb;
  hb.temp = (float)T;
  hb.k0 = (uint32_t)seed;
  hb.k1 = (uint32_t)(seed >> 32);
  hb.sweep = (uint32_t)sweep;
  gf_status st;
  for (int p = 0; p < 2; ++p)
    if ((st = update_tracked(c, U, Gx, g, gauge, p, hb, "tracked heatbath")) != GF_OK) return st;
  UpdMicro<float> mc;
  for (int k = 0; k < n_micro; ++k)
    for (int p = 0; p < 2; ++p)
      if ((st = update_tracked(c, U, Gx, g, gauge, p, mc, "tracked microcanonical")) != GF_OK) return st;
  return GF_OK;
}

gf_status gf_heatbath_half_tracked(gf_ctx* c, void* U, void* G, const gf_geom* g, int32_t gauge,
                                   int32_t parity, double T, uint64_t seed, uint64_t sweep) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_heatbath_half_tracked");
  CHECK_GAUGE_PARITY(c, gauge, parity, "gf_heatbath_half_tracked");
  REJECT_MAG(c, gauge, "gf_heatbath_half_tracked");
  CHECK_TRACKED(c, U, G, g, "gf_heatbath_half_tracked");
  if (!(T > 0.0) || !std::isfinite(T))
    return fail(c, GF_ERR_ARG, "gf_heatbath_half_tracked: T must be > 0");
  UpdHB<float> hb;
  hb.temp = (float)T;
  hb.k0 = (uint32_t)seed;
  hb.k1 = (uint32_t)(seed >> 32);
  hb.sweep = (uint32_t)sweep;
  return update_tracked(c, U, G, g, gauge, parity, hb, "gf_heatbath_half_tracked");
}

gf_status gf_micro_half_tracked(gf_ctx* c, void* U, void* G, const gf_geom* g, int32_t gauge,
                                int32_t parity) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_micro_half_tracked");
  CHECK_GAUGE_PARITY(c, gauge, parity, "gf_micro_half_tracked");
  REJECT_MAG(c, gauge, "gf_micro_half_tracked");
  CHECK_TRACKED(c, U, G, g, "gf_micro_half_tracked");
  return update_tracked(c, U, G, g, gauge, parity, UpdMicro<float>(), "gf_micro_half_tracked");
}
