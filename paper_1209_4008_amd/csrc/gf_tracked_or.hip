// gf_tracked_or.hip -- FP32 overrelaxation half-sweeps with the site
// transformations accumulated into a gauge-transformation field.
#include "gf_host.hpp"

gf_status sweep_tracked(gf_ctx* c, void* U, void* Gx, const gf_geom* g, int32_t gauge,
                               int32_t parity, double omega) {
  UpdOR<float> upd;
  upd.omega = (float)omega;
  return update_tracked(c, U, Gx, g, gauge, parity, upd, "tracked overrelaxation");
}

gf_status sweep_form_tracked(gf_ctx* c, void* U, void* Gx, const gf_geom* g,
                                    int32_t gauge, int32_t parity, double omega, int32_t form) {
  if (form == 0) return sweep_tracked(c, U, Gx, g, gauge, parity, omega);
  UpdORForm<float> upd;
  upd.omega = (float)omega;
  upd.form = form;
  return update_tracked(c, U, Gx, g, gauge, parity, upd, "tracked overrelaxation (form)");
}

gf_status gf_sweep_tracked(gf_ctx* c, void* U, void* G, const gf_geom* g, int32_t gauge,
                           int32_t parity, double omega) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_sweep_tracked");
  CHECK_GAUGE_PARITY(c, gauge, parity, "gf_sweep_tracked");
  CHECK_TRACKED(c, U, G, g, "gf_sweep_tracked");
  if (!(omega >= 1.0 && omega < 2.0))
    return fail(c, GF_ERR_ARG, "gf_sweep_tracked: omega must be in [1, 2)");
  return sweep_tracked(c, U, G, g, gauge, parity, omega);
}
