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
