// gf_sweep_form.hip -- overrelaxation half-sweeps with the other forms of
// g^omega (gf_sweep_form).
#include "gf_host.hpp"

gf_status gf_sweep_form(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, int32_t parity,
                        double omega, int32_t form) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_sweep_form");
  CHECK_GAUGE_PARITY(c, gauge, parity, "gf_sweep_form");
  if (!U) return fail(c, GF_ERR_ARG, "gf_sweep_form: NULL field");
  if (!(omega >= 1.0 && omega < 2.0))
    return fail(c, GF_ERR_ARG, "gf_sweep_form: omega must be in [1, 2)");
  if (form < 0 || form > 3) return fail(c, GF_ERR_ARG, "gf_sweep_form: form must be 0..3");
  if (form == 0) return gf_sweep(c, U, g, gauge, parity, omega);
  return launch_update(
      c, U, g, gauge, parity,
      [&]<typename T>() {
        UpdORForm<T> u;
        u.omega = (T)omega;
        u.form = form;
        return u;
      },
      "gf_sweep_form");
}
