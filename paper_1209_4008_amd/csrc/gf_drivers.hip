// gf_drivers.hip -- the gauge-fixing drivers gf_fix and gf_fix_mixed.
#include "gf_driver.hpp"

using namespace gfdrv;

namespace {

gf_status run_anneal(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, const gf_fix_params* p,
                     Timer& tm, int32_t* done, void* Gx = nullptr) {
  gf_status st;
  *done = 0;
  for (int32_t k = 0; k < p->sa_steps; ++k) {
    const double T = p->sa_steps > 1
                         ? p->sa_T0 + (p->sa_T1 - p->sa_T0) * (double)k / (double)(p->sa_steps - 1)
                         : p->sa_T0;
    if ((st = tm.begin()) != GF_OK) return st;
    st = Gx ? anneal_step_tracked(c, U, Gx, g, gauge, T, p->seed, (uint64_t)k, p->sa_micro)
            : gf_anneal_sweep(c, U, g, gauge, T, p->seed, (uint64_t)k, p->sa_micro);
    if (st != GF_OK) return st;
    if ((st = tm.end(4, 2 + 2 * (int64_t)p->sa_micro)) != GF_OK) return st;
    if (p->sa_reunit_every > 0 && (k + 1) % p->sa_reunit_every == 0)
      if ((st = gf_reunitarize(c, U, g)) != GF_OK) return st;
    *done = k + 1;
  }
  return GF_OK;
}

// reunitarise (optional), measure F and theta, copy to the host
gf_status do_check(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, bool reunit, Timer& tm,
                   Phase& ph, CheckLog& log) {
  gf_status st;
  const int nout = gauge == GF_COULOMB ? g->nt : 1;
  if ((st = ensure_out(c, nout)) != GF_OK) return st;
  if (log.monitor()) {
    // the drift the sweeps left, before the reunitarisation removes it
    if ((st = ensure_mon(c)) != GF_OK) return st;
    if ((st = tm.begin()) != GF_OK) return st;
    if ((st = unitarity_launch(c, U, g, c->dev_mon)) != GF_OK) return st;
    if ((st = tm.end(2, 2)) != GF_OK) return st;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->host_mon, c->dev_mon, sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
  }
  if (reunit) {
    if ((st = tm.begin()) != GF_OK) return st;
    if ((st = gf_reunitarize(c, U, g)) != GF_OK) return st;
    if ((st = tm.end(3, 1)) != GF_OK) return st;
  }
  if ((st = tm.begin()) != GF_OK) return st;
  if ((st = measure_impl(c, U, g, gauge, c->dev_out, c->dev_out + c->out_cap)) != GF_OK) return st;
  if ((st = tm.end(2, 2)) != GF_OK) return st;
  HIP_OR_FAIL(c, hipMemcpyAsync(c->host_out, c->dev_out, 2 * c->out_cap * sizeof(double),
                                hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if ((st = tm.flush()) != GF_OK) return st;
  double Fsum = 0, thmax = 0;
  for (int t = 0; t < nout; ++t) {
    const double F = c->host_out[t], th = c->host_out[c->out_cap + t];
    if (!std::isfinite(F) || !std::isfinite(th))
      return fail(c, GF_ERR_NONFINITE, "gf_fix: non-finite F or theta after %d sweeps", ph.sweeps);
    Fsum += F;
    thmax = th > thmax ? th : thmax;
  }
  ph.F = Fsum / nout;
  ph.theta = thmax;
  ph.checks++;
  log.record(ph.sweeps, g->prec, ph.F, ph.theta, log.monitor() ? c->host_mon[0] : -1);
  return GF_OK;
}

// enqueue n sweeps (RED then BLACK each) on the context stream; with
// stochastic relaxation (p->sr_prob > 0) the draws of sweep first + k use
// sweep index first + k
gf_status enqueue_sweeps(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge,
                         const gf_fix_params* p, int32_t n, void* Gx, int32_t first) {
  gf_status st;
  const bool sr = p->sr_prob > 0.0;
  for (int32_t k = 0; k < n; ++k)
    for (int par = 0; par < 2; ++par) {
      const uint64_t sw = (uint64_t)(first + k);
      if (sr)
        st = Gx ? sweep_sr_tracked(c, U, Gx, g, gauge, par, p->omega, p->sr_prob, p->seed, sw)
                : gf_sweep_sr(c, U, g, gauge, par, p->omega, p->sr_prob, p->seed, sw);
      else
        st = Gx ? sweep_form_tracked(c, U, Gx, g, gauge, par, p->omega, p->or_form)
                : gf_sweep_form(c, U, g, gauge, par, p->omega, p->or_form);
      if (st != GF_OK) return st;
    }
  return GF_OK;
}

gf_status capture_sweeps(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge,
                         const gf_fix_params* p, int32_t n, void* Gx, SweepGraph& sg) {
  if (!c->capture) HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
  hipStream_t saved = c->stream;
  c->stream = c->capture;
  hipError_t e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal);
  gf_status st = GF_OK;
  if (e != hipSuccess) {
    c->stream = saved;
    return fail(c, GF_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  st = enqueue_sweeps(c, U, g, gauge, p, n, Gx, 0);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(c->capture, &graph);
  c->stream = saved;
  if (st != GF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(c, GF_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  sg.graph = graph;
  HIP_OR_FAIL(c, hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0));
  sg.n = n;
  return GF_OK;
}

// sets the context's timeslice mask for the lifetime of a driver phase
struct MaskScope {
  gf_ctx* c;
  explicit MaskScope(gf_ctx* ctx, const uint8_t* m) : c(ctx) { c->tmask = m; }
  ~MaskScope() { c->tmask = nullptr; }
};

// Coulomb with GF_FLAG_FREEZE_TIMESLICES: after a check, freeze every
// timeslice whose theta_t (host_out, as do_check left it) is below target;
// returns the number still active and uploads the mask when it changed
gf_status update_tmask(gf_ctx* c, const gf_geom* g, double target, int* n_active) {
  bool changed = false;
  int n = 0;
  for (int t = 0; t < g->nt; ++t) {
    if (c->host_tmask[t] && c->host_out[c->out_cap + t] < target) {
      c->host_tmask[t] = 0;
      changed = true;
    }
    n += c->host_tmask[t];
  }
  // the previous upload has completed: do_check synchronised the stream
  if (changed && n > 0)
    HIP_OR_FAIL(c, hipMemcpyAsync(c->dev_tmask, c->host_tmask, (size_t)g->nt,
                                  hipMemcpyHostToDevice, c->stream));
  *n_active = n;
  return GF_OK;
}

// sweeps `geom`'s field until theta < target or max_sweeps; with
// GF_FLAG_FREEZE_TIMESLICES (Coulomb) until every timeslice has had
// theta_t < target at a check, each timeslice frozen from that check on
gf_status run_phase(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, const gf_fix_params* p,
                    double target, bool first_check_reunit, Timer& tm, Phase& ph, CheckLog& log,
                    void* Gx = nullptr) {
  gf_status st;
  const int cat = g->prec == GF_FP32 ? 0 : 1;
  // stochastic relaxation changes its kernel arguments every sweep: no replay
  const bool use_graph = (p->flags & GF_FLAG_GRAPH) != 0 && !(p->sr_prob > 0.0);
  const bool freeze = gauge == GF_COULOMB && (p->flags & GF_FLAG_FREEZE_TIMESLICES) != 0;
  if (freeze) {
    if ((st = ensure_tmask(c, (size_t)g->nt)) != GF_OK) return st;
    memset(c->host_tmask, 1, (size_t)g->nt);
    HIP_OR_FAIL(c, hipMemcpyAsync(c->dev_tmask, c->host_tmask, (size_t)g->nt,
                                  hipMemcpyHostToDevice, c->stream));
  }
  MaskScope scope(c, freeze ? c->dev_tmask : nullptr);
  SweepGraph sg;
  int n_active = g->nt;
  for (;;) {
    const bool reunit = p->reunit_at_check && (ph.sweeps > 0 || first_check_reunit);
    if ((st = do_check(c, U, g, gauge, reunit, tm, ph, log)) != GF_OK) return st;
    if (freeze) {
      if ((st = update_tmask(c, g, target, &n_active)) != GF_OK) return st;
      if (n_active == 0) {
        ph.converged = 1;
        return GF_OK;
      }
    } else if (ph.theta < target) {
      ph.converged = 1;
      return GF_OK;
    }
    if (ph.sweeps >= p->max_sweeps) return GF_OK;
    const int32_t n = std::min(p->check_every, p->max_sweeps - ph.sweeps);
    if (use_graph && n == p->check_every && !sg.exec)
      if ((st = capture_sweeps(c, U, g, gauge, p, n, Gx, sg)) != GF_OK) return st;
    if ((st = tm.begin()) != GF_OK) return st;
    if (use_graph && sg.exec && n == sg.n)
      HIP_OR_FAIL(c, hipGraphLaunch(sg.exec, c->stream));
    else if ((st = enqueue_sweeps(c, U, g, gauge, p, n, Gx, ph.sweeps)) != GF_OK)
      return st;
    if ((st = tm.end(cat, 2 * (int64_t)n)) != GF_OK) return st;
    ph.sweeps += n;
    ph.skipped += (int64_t)(g->nt - n_active) * n;
  }
}

}  // namespace

gf_status gf_fix(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge, const gf_fix_params* p,
                 gf_fix_result* r) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_fix");
  if (gauge != GF_LANDAU && gauge != GF_COULOMB && gauge != GF_MAG)
    return fail(c, GF_ERR_ARG, "gf_fix: bad gauge");
  if (gauge == GF_MAG && p && (p->sa_steps > 0 || p->sr_prob > 0.0))
    return fail(c, GF_ERR_UNSUPPORTED, "gf_fix: annealing and stochastic relaxation are not "
                                       "available for GF_MAG");
  if (!U || !r) return fail(c, GF_ERR_ARG, "gf_fix: NULL pointer");
  gf_status st = check_params(c, p);
  if (st != GF_OK) return st;
  if ((p->flags & GF_FLAG_FREEZE_TIMESLICES) && gauge != GF_COULOMB)
    return fail(c, GF_ERR_ARG, "gf_fix: GF_FLAG_FREEZE_TIMESLICES needs GF_COULOMB");
  init_result(r);
  const auto t0 = std::chrono::steady_clock::now();
  Timer tm{c, (p->flags & GF_FLAG_TIMING) != 0, r->kernel_ms, r->kernel_launches};
  Phase ph;
  CheckLog log{p, r, t0};
  st = run_anneal(c, U, g, gauge, p, tm, &r->sa_steps);
  if (st == GF_OK) st = run_phase(c, U, g, gauge, p, p->theta_target, false, tm, ph, log);
  if (st == GF_OK) st = tm.flush();
  r->sweeps = ph.sweeps;
  r->checks = ph.checks;
  r->F = ph.F;
  r->theta = ph.theta;
  r->frozen_slice_sweeps = clamp_i32(ph.skipped);
  r->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st != GF_OK) {
    r->status = st;
    return st;
  }
  r->status = ph.converged ? GF_OK : GF_NOT_CONVERGED;
  return r->status;
}

gf_status gf_fix_mixed(gf_ctx* c, void* U_lo, const gf_geom* g_lo, void* U_hi,
                       const gf_geom* g_hi, int32_t gauge, const gf_fix_params* p,
                       gf_fix_result* r) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g_lo, "gf_fix_mixed(lo)");
  CHECK_GEOM(c, g_hi, "gf_fix_mixed(hi)");
  if (g_lo->prec != GF_FP32 || g_hi->prec != GF_FP64)
    return fail(c, GF_ERR_ARG, "gf_fix_mixed: needs an FP32 and an FP64 field");
  if (!same_extents(g_lo, g_hi)) return fail(c, GF_ERR_ARG, "gf_fix_mixed: extents differ");
  if (gauge != GF_LANDAU && gauge != GF_COULOMB && gauge != GF_MAG)
    return fail(c, GF_ERR_ARG, "gf_fix_mixed: bad gauge");
  if (gauge == GF_MAG && p && (p->sa_steps > 0 || p->sr_prob > 0.0))
    return fail(c, GF_ERR_UNSUPPORTED, "gf_fix_mixed: annealing and stochastic relaxation are "
                                       "not available for GF_MAG");
  if (!U_lo || !U_hi || !r) return fail(c, GF_ERR_ARG, "gf_fix_mixed: NULL pointer");
  {
    const char *a = (const char*)U_lo, *b = (const char*)U_hi;
    if (a < b + gf_field_bytes(g_hi) && b < a + gf_field_bytes(g_lo))
      return fail(c, GF_ERR_ARG, "gf_fix_mixed: buffers overlap");
  }
  gf_status st = check_params(c, p);
  if (st != GF_OK) return st;
  if (!(p->theta_switch > 0.0)) return fail(c, GF_ERR_ARG, "gf_fix_mixed: theta_switch must be > 0");
  if ((p->flags & GF_FLAG_FREEZE_TIMESLICES) && gauge != GF_COULOMB)
    return fail(c, GF_ERR_ARG, "gf_fix_mixed: GF_FLAG_FREEZE_TIMESLICES needs GF_COULOMB");
  const bool track = (p->flags & GF_FLAG_NO_TRACK) == 0;
  const Lat L = make_lat(g_lo);
  if (track) {
    const size_t gbytes = (size_t)2 * L.vp * 6 * sizeof(float) * 2;
    if (gbytes > c->gbuf_cap) {
      if (c->gbuf) HIP_OR_FAIL(c, hipFree(c->gbuf));
      c->gbuf = nullptr;
      c->gbuf_cap = 0;
      HIP_OR_FAIL(c, hipMalloc(&c->gbuf, gbytes));
      c->gbuf_cap = gbytes;
    }
  }
  init_result(r);
  const auto t0 = std::chrono::steady_clock::now();
  Timer tm{c, (p->flags & GF_FLAG_TIMING) != 0, r->kernel_ms, r->kernel_launches};
  Phase lo, hi;
  CheckLog log{p, r, t0};
  // FP64 input -> FP32 working copy; g = 1
  if ((st = tm.begin()) == GF_OK && (st = gf_convert(c, g_hi, U_hi, g_lo, U_lo, 0)) == GF_OK) {
    if (track)
      hipLaunchKernelGGL((k_fill_unit<float, 6, 1>), dim3(blocks_for(L.vp), 2), dim3(kBlock), 0,
                         c->stream, (v2<float>*)c->gbuf, L.vp);
    st = launch_check(c, "gf_fix_mixed: init");
    if (st == GF_OK) st = tm.end(3, track ? 2 : 1);
  }
  if (st == GF_OK) st = run_anneal(c, U_lo, g_lo, gauge, p, tm, &r->sa_steps, track ? c->gbuf : nullptr);
  if (st == GF_OK)
    st = run_phase(c, U_lo, g_lo, gauge, p, p->theta_switch, false, tm, lo, log,
                   track ? c->gbuf : nullptr);
  if (st == GF_OK) {
    r->theta_at_switch = lo.theta;
    // back to FP64: either the original field transformed by g (projected onto
    // SU(3) in FP64), or the FP32 field itself reunitarised in FP64
    if ((st = tm.begin()) == GF_OK) {
      if (track) {
        with_type(g_hi, [&]<typename T, int NC>() {
          hipLaunchKernelGGL((k_apply_gauge<T, NC, float>), dim3(blocks_for(L.vh), 2), dim3(kBlock),
                             0, c->stream, (v2<T>*)U_hi, (const v2<float>*)c->gbuf, L);
        });
        st = launch_check(c, "gf_fix_mixed: apply g");
      } else {
        st = gf_convert(c, g_lo, U_lo, g_hi, U_hi, 1);
      }
    }
    if (st == GF_OK) st = tm.end(3, 1);
    if (st == GF_OK) st = run_phase(c, U_hi, g_hi, gauge, p, p->theta_target, false, tm, hi, log);
  }
  if (st == GF_OK) st = tm.flush();
  r->sweeps_lo = lo.sweeps;
  r->sweeps = lo.sweeps + hi.sweeps;
  r->checks = lo.checks + hi.checks;
  r->F = hi.checks ? hi.F : lo.F;
  r->theta = hi.checks ? hi.theta : lo.theta;
  r->frozen_slice_sweeps = clamp_i32(lo.skipped + hi.skipped);
  r->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st != GF_OK) {
    r->status = st;
    return st;
  }
  r->status = hi.converged ? GF_OK : GF_NOT_CONVERGED;
  return r->status;
}
