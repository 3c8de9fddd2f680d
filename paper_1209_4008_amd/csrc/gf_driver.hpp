// gf_driver.hpp -- pieces shared by the gauge-fixing drivers and the batch
// driver: kernel timing on event pairs, the captured sweep block, parameter
// validation and result initialisation.
#pragma once

#include "gf_host.hpp"

namespace gfdrv {


// Kernel timing of the drivers: each timed interval records a pair of pool
// events on the context stream; elapsed times are read at the driver's own
// synchronisation points (flush), so timing adds no host waits.
struct Timer {
  gf_ctx* c;
  bool on;
  double* ms;
  int64_t* n;
  struct Pending {
    int cat;
    int64_t launches;
  };
  std::vector<Pending> pending;
  size_t used = 0;  // events of the pool in use
  gf_status begin() {
    if (!on) return GF_OK;
    while (c->pool.size() < used + 2) {
      hipEvent_t e;
      HIP_OR_FAIL(c, hipEventCreate(&e));
      c->pool.push_back(e);
    }
    HIP_OR_FAIL(c, hipEventRecord(c->pool[used], c->stream));
    return GF_OK;
  }
  gf_status end(int cat, int64_t launches) {
    if (!on) return GF_OK;
    HIP_OR_FAIL(c, hipEventRecord(c->pool[used + 1], c->stream));
    used += 2;
    pending.push_back({cat, launches});
    if (used >= 4096) return flush();
    return GF_OK;
  }
  // waits for the last recorded event and adds up the pending intervals
  gf_status flush() {
    if (!on || pending.empty()) return GF_OK;
    HIP_OR_FAIL(c, hipEventSynchronize(c->pool[used - 1]));
    for (size_t k = 0; k < pending.size(); ++k) {
      float t = 0;
      HIP_OR_FAIL(c, hipEventElapsedTime(&t, c->pool[2 * k], c->pool[2 * k + 1]));
      ms[pending[k].cat] += t;
      n[pending[k].cat] += pending[k].launches;
    }
    pending.clear();
    used = 0;
    return GF_OK;
  }
};

struct Phase {
  int32_t sweeps = 0;
  int32_t checks = 0;
  int converged = 0;
  double F = 0, theta = 0;
  int64_t skipped = 0;  // timeslice-sweeps not done (frozen timeslices)
};

inline gf_status check_params(gf_ctx* c, const gf_fix_params* p) {
  if (!p) return fail(c, GF_ERR_ARG, "gf_fix: NULL params");
  if (!(p->omega >= 1.0 && p->omega < 2.0)) return fail(c, GF_ERR_ARG, "gf_fix: omega must be in [1, 2)");
  if (p->max_sweeps < 0 || p->check_every < 1) return fail(c, GF_ERR_ARG, "gf_fix: bad sweep counts");
  if (!(p->theta_target >= 0.0)) return fail(c, GF_ERR_ARG, "gf_fix: bad theta_target");
  if (p->sa_steps < 0 || p->sa_micro < 0 || p->sa_reunit_every < 0)
    return fail(c, GF_ERR_ARG, "gf_fix: bad annealing parameters");
  if (p->check_log && p->check_log_cap < 0) return fail(c, GF_ERR_ARG, "gf_fix: bad check_log_cap");
  if (p->or_form < 0 || p->or_form > 3) return fail(c, GF_ERR_ARG, "gf_fix: or_form must be 0..3");
  if (p->or_form != 0 && p->sr_prob > 0.0)
    return fail(c, GF_ERR_UNSUPPORTED, "gf_fix: or_form != 0 with stochastic relaxation");
  if (!(p->sr_prob >= 0.0 && p->sr_prob <= 1.0))
    return fail(c, GF_ERR_ARG, "gf_fix: sr_prob must be in [0, 1]");
  if (p->sa_steps > 0 && (!(p->sa_T0 > 0.0) || !(p->sa_T1 > 0.0) || !std::isfinite(p->sa_T0) ||
                          !std::isfinite(p->sa_T1)))
    return fail(c, GF_ERR_ARG, "gf_fix: annealing temperatures must be > 0");
  return GF_OK;
}



// a captured block of n sweeps, replayed between checks
struct SweepGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t n = 0;
  SweepGraph() = default;
  SweepGraph(const SweepGraph&) = delete;
  SweepGraph& operator=(const SweepGraph&) = delete;
  // drop the captured block (its launches name tables or shapes that changed)
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    n = 0;
  }
  ~SweepGraph() { reset(); }
};

inline void init_result(gf_fix_result* r) {
  memset(r, 0, sizeof *r);
  r->unitarity_max = -1;
}

// what a driver records at its checks: the unitarity monitor (GF_FLAG_MONITOR)
// and the caller's check log (params.check_log), both into the result
struct CheckLog {
  const gf_fix_params* p;
  gf_fix_result* r;
  std::chrono::steady_clock::time_point t0;
  bool monitor() const { return (p->flags & GF_FLAG_MONITOR) != 0; }
  void record(int32_t sweeps, int32_t prec, double F, double theta, double unitarity) {
    if (monitor() && unitarity > r->unitarity_max) r->unitarity_max = unitarity;
    if (!p->check_log || r->check_log_n >= p->check_log_cap) return;
    gf_check_record& e = p->check_log[r->check_log_n++];
    e.sweeps = sweeps;
    e.prec = prec;
    e.F = F;
    e.theta = theta;
    e.unitarity = monitor() ? unitarity : -1;
    e.elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

inline int32_t clamp_i32(int64_t v) { return v > INT32_MAX ? INT32_MAX : (int32_t)v; }

}  // namespace gfdrv
