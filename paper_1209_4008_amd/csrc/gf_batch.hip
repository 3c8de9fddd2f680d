// gf_batch.hip -- batches of independent lattices (Gribov copies, uneven
// extents) fixed together.
#include "gf_driver.hpp"

using namespace gfdrv;

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
struct gf_batch {
  gf_ctx* c = nullptr;
  int n = 0;
  int storage = GF_R12;
  std::vector<gf_geom> g64, g32;  // caller's FP64 geometries, FP32 12-real working ones
  std::vector<void*> U64;         // caller's fields
  std::vector<Lat> lat;
  void* arena32 = nullptr;  // FP32 working fields
  void* arenaG = nullptr;   // gauge-transformation fields
  std::vector<size_t> off32, offG;
  std::vector<int> active;  // lattices still in the current phase
  double* d_out = nullptr;  // F[n], theta[n]
  double* h_out = nullptr;  // pinned
  double* d_partial = nullptr;
  size_t partial_cap = 0;
  void* d_tab = nullptr;  // scratch for the lattice tables (4 tables)
  size_t tab_cap = 0;
  uint32_t* d_map[4] = {nullptr, nullptr, nullptr, nullptr};  // their block maps
  size_t map_cap[4] = {0, 0, 0, 0};                           // entries
};

namespace {

// A batch launch sweeps the fields of all the lattices still active, so with
// no variant set on the context its built-in mode follows their total size
// (the 192-lattice batch, 10.8 GB in FP64 12-real: streamed 5.25 against
// cached 4.73 TB/s).
size_t active_bytes(const gf_batch* b, bool lo) {
  const std::vector<gf_geom>& gs = lo ? b->g32 : b->g64;
  size_t total = 0;
  for (int l = 0; l < b->n; ++l)
    if (b->active[l]) total += gf_field_bytes(&gs[l]);
  return total;
}
int batch_nt(const gf_ctx* c, const gf_batch* b, bool lo, int kind) {
  const gf_geom& g = lo ? b->g32[0] : b->g64[0];
  return ctx_nt_bytes(c, &g, kind, active_bytes(b, lo));
}
int batch_tps(const gf_ctx* c, const gf_batch* b, bool lo, int kind) {
  const gf_geom& g = lo ? b->g32[0] : b->g64[0];
  return ctx_tps_bytes(c, &g, kind, active_bytes(b, lo));
}

template <typename T>
struct TableSet {
  std::vector<BatchEntry<T>> h;
  std::vector<uint32_t> map;  // table entry of each block
  uint32_t blocks = 0;
};

// table of the active lattices for one launch shape (threads per lattice =
// vh * tps)
template <typename T>
TableSet<T> make_table(const gf_batch* b, bool lo, int tps) {
  TableSet<T> t;
  uint32_t blk = 0;
  for (int l = 0; l < b->n; ++l) {
    if (!b->active[l]) continue;
    BatchEntry<T> e;
    e.L = b->lat[l];
    e.U = lo ? (v2<T>*)((char*)b->arena32 + b->off32[l]) : (v2<T>*)b->U64[l];
    e.Gx = lo ? (v2<T>*)((char*)b->arenaG + b->offG[l]) : nullptr;
    e.first_block = blk;
    e.index = (uint32_t)l;
    const uint32_t nb = blocks_for((uint64_t)e.L.vh * (uint64_t)tps);
    t.map.insert(t.map.end(), nb, (uint32_t)t.h.size());
    blk += nb;
    t.h.push_back(e);
  }
  t.blocks = blk;
  return t;
}

struct BatchPhase {
  std::vector<int32_t> sweeps, checks, converged;
  std::vector<double> F, theta;
};

}  // namespace

gf_status gf_batch_create(gf_ctx* c, int32_t n, const gf_geom* geoms, void* const* U,
                          int32_t gauge, gf_batch** out) {
  CHECK_CTX(c);
  if (!out || n < 1 || !geoms || !U) return fail(c, GF_ERR_ARG, "gf_batch_create: bad arguments");
  *out = nullptr;
  if (gauge != GF_LANDAU) return fail(c, GF_ERR_UNSUPPORTED, "gf_batch_create: Landau batches only");
  for (int l = 0; l < n; ++l) {
    if (!geom_ok(&geoms[l]) || geoms[l].prec != GF_FP64 || geoms[l].storage != geoms[0].storage || !U[l])
      return fail(c, GF_ERR_ARG, "gf_batch_create: lattice %d: needs a valid FP64 geometry of the "
                                 "common storage and a field", l);
  }
  gf_batch* b = new gf_batch();
  b->c = c;
  b->n = n;
  b->storage = geoms[0].storage;
  size_t s32 = 0, sG = 0;
  for (int l = 0; l < n; ++l) {
    b->g64.push_back(geoms[l]);
    gf_geom g = geoms[l];
    g.prec = GF_FP32;
    g.storage = GF_R12;
    b->g32.push_back(g);
    b->U64.push_back(U[l]);
    b->lat.push_back(make_lat(&geoms[l]));
    b->off32.push_back(s32);
    b->offG.push_back(sG);
    s32 += (gf_field_bytes(&g) + 255) / 256 * 256;
    sG += ((size_t)b->lat[l].vp * 2 * 6 * 2 * sizeof(float) + 255) / 256 * 256;
  }
  auto cleanup = [&](gf_status st, const char* what) {
    gf_batch_destroy(b);
    return fail(c, st, "gf_batch_create: %s", what);
  };
  if (hipMalloc(&b->arena32, s32) != hipSuccess) return cleanup(GF_ERR_NOMEM, "FP32 fields");
  if (hipMalloc(&b->arenaG, sG) != hipSuccess) return cleanup(GF_ERR_NOMEM, "g fields");
  b->active.assign(n, 1);
  if (hipMalloc(&b->d_out, 2 * n * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&b->h_out, 2 * n * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return cleanup(GF_ERR_NOMEM, "control buffers");
  *out = b;
  return GF_OK;
}

gf_status gf_batch_destroy(gf_batch* b) {
  if (!b) return GF_ERR_ARG;
  if (b->c) (void)hipSetDevice(b->c->device);
  if (b->arena32) (void)hipFree(b->arena32);
  if (b->arenaG) (void)hipFree(b->arenaG);
  if (b->d_out) (void)hipFree(b->d_out);
  if (b->h_out) (void)hipHostFree(b->h_out);
  if (b->d_partial) (void)hipFree(b->d_partial);
  if (b->d_tab) (void)hipFree(b->d_tab);
  for (int k = 0; k < 4; ++k)
    if (b->d_map[k]) (void)hipFree(b->d_map[k]);
  delete b;
  return GF_OK;
}

namespace {

// upload a table and its block map into slot k of the batch's scratch;
// returns their device addresses
template <typename T>
gf_status upload_table(gf_batch* b, int k, const TableSet<T>& t, const BatchEntry<T>** dev,
                       const uint32_t** dev_map) {
  gf_ctx* c = b->c;
  const size_t one = ((size_t)b->n * sizeof(BatchEntry<T>) + 255) / 256 * 256;
  if (b->tab_cap < 4 * one) {
    if (b->d_tab) HIP_OR_FAIL(c, hipFree(b->d_tab));
    b->d_tab = nullptr;
    b->tab_cap = 0;
    HIP_OR_FAIL(c, hipMalloc(&b->d_tab, 4 * one));
    b->tab_cap = 4 * one;
  }
  char* p = (char*)b->d_tab + (size_t)k * one;
  // kernels still queued on the context stream may read this slot (the
  // context stream need not be the null stream that hipMemcpy orders with)
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  HIP_OR_FAIL(c, hipMemcpy(p, t.h.data(), t.h.size() * sizeof(BatchEntry<T>), hipMemcpyHostToDevice));
  *dev = (const BatchEntry<T>*)p;
  if (t.map.size() > b->map_cap[k]) {
    if (b->d_map[k]) HIP_OR_FAIL(c, hipFree(b->d_map[k]));
    b->d_map[k] = nullptr;
    b->map_cap[k] = 0;
    HIP_OR_FAIL(c, hipMalloc(&b->d_map[k], t.map.size() * sizeof(uint32_t)));
    b->map_cap[k] = t.map.size();
  }
  HIP_OR_FAIL(c, hipMemcpy(b->d_map[k], t.map.data(), t.map.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice));
  *dev_map = b->d_map[k];
  return GF_OK;
}

template <typename T, int NC, class Upd, bool TRACK>
void launch_batch_update(gf_ctx* c, int tps, int nt, const BatchEntry<T>* tab,
                         const uint32_t* map, uint32_t blocks, int parity, const Upd& upd) {
  auto go = [&]<int TPS, int NT>() {
    hipLaunchKernelGGL((k_update_half_batch<T, NC, Upd, TPS, NT, TRACK>), dim3(blocks), dim3(kBlock),
                       0, c->stream, tab, map, parity, upd);
  };
  auto go_tps = [&]<int NT>() {
    if (tps == 1) go.template operator()<1, NT>();
    else if (tps == 2) go.template operator()<2, NT>();
    else go.template operator()<4, NT>();
  };
  const int mode = nt_mode<Upd>(nt);
  if (mode == kNTAll) {
    go_tps.template operator()<kNTAll>();
  } else if (mode == kNTStores) {
    if constexpr (HasStoreMode<Upd>::value) go_tps.template operator()<kNTStores>();
  } else {
    go_tps.template operator()<kNTNone>();
  }
}

// the launch tables of one phase over the active lattices: the sweep table
// (tps lanes per site) and the measurement table (one thread per half index)
template <typename T>
struct PhaseTables {
  TableSet<T> sweep, meas;
  const BatchEntry<T>* d_sweep = nullptr;
  const BatchEntry<T>* d_meas = nullptr;
  const uint32_t* d_sweep_map = nullptr;
  const uint32_t* d_meas_map = nullptr;
  int n = 0;    // entries (active lattices)
  int tps = 1;  // lanes per site and nontemporal mode for their total size
  int nt = 0;
};

template <typename T>
gf_status build_tables(gf_batch* b, bool lo, int kind, PhaseTables<T>& pt) {
  pt.tps = batch_tps(b->c, b, lo, kind);
  pt.nt = batch_nt(b->c, b, lo, kind);
  pt.sweep = make_table<T>(b, lo, pt.tps);
  pt.meas = make_table<T>(b, lo, 1);
  pt.n = (int)pt.sweep.h.size();
  gf_status st;
  if (pt.n == 0) return GF_OK;
  if ((st = upload_table(b, lo ? 0 : 2, pt.sweep, &pt.d_sweep, &pt.d_sweep_map)) != GF_OK) return st;
  return upload_table(b, lo ? 1 : 3, pt.meas, &pt.d_meas, &pt.d_meas_map);
}

// one batch phase (precision T, storage NC): checks and sweeps until every
// lattice has theta < target or max_sweeps. A lattice leaves the phase at the
// check that finds it converged (or out of sweeps); the tables are then
// rebuilt over the lattices still active and the sweep block recaptured, so
// that no launch covers a lattice that has left.
template <typename T, int NC>
gf_status batch_phase(gf_batch* b, const gf_fix_params* p, bool lo, double target, Timer& tm,
                      BatchPhase& ph) {
  gf_ctx* c = b->c;
  const int n = b->n;
  b->active.assign(n, 1);
  PhaseTables<T> pt;
  gf_status st;
  if ((st = build_tables(b, lo, kSweepKind, pt)) != GF_OK) return st;
  const size_t need = 2 * (size_t)pt.meas.blocks;
  if (need > b->partial_cap) {
    if (b->d_partial) HIP_OR_FAIL(c, hipFree(b->d_partial));
    b->d_partial = nullptr;
    b->partial_cap = 0;
    HIP_OR_FAIL(c, hipMalloc(&b->d_partial, need * sizeof(double)));
    b->partial_cap = need;
  }
  ph.sweeps.assign(n, 0);
  ph.checks.assign(n, 0);
  ph.converged.assign(n, 0);
  ph.F.assign(n, 0.0);
  ph.theta.assign(n, 0.0);
  UpdOR<T> upd;
  upd.omega = (T)p->omega;
  const bool sr = p->sr_prob > 0.0;
  const bool use_graph = (p->flags & GF_FLAG_GRAPH) != 0 && !sr;
  SweepGraph sg;
  int32_t done = 0;  // sweeps done by the lattices still active
  auto enqueue = [&](int32_t nsw) {
    for (int32_t k = 0; k < nsw; ++k)
      for (int par = 0; par < 2; ++par) {
        if (sr) {
          UpdSR<T> us;
          us.omega = (T)p->omega;
          us.prob = p->sr_prob;
          us.k0 = (uint32_t)p->seed;
          us.k1 = (uint32_t)(p->seed >> 32);
          us.sweep = (uint32_t)(done + k);
          if (lo)
            launch_batch_update<T, NC, UpdSR<T>, true>(c, pt.tps, pt.nt, pt.d_sweep, pt.d_sweep_map, pt.sweep.blocks, par, us);
          else
            launch_batch_update<T, NC, UpdSR<T>, false>(c, pt.tps, pt.nt, pt.d_sweep, pt.d_sweep_map, pt.sweep.blocks, par, us);
        } else if (lo) {
          launch_batch_update<T, NC, UpdOR<T>, true>(c, pt.tps, pt.nt, pt.d_sweep, pt.d_sweep_map, pt.sweep.blocks, par, upd);
        } else {
          launch_batch_update<T, NC, UpdOR<T>, false>(c, pt.tps, pt.nt, pt.d_sweep, pt.d_sweep_map, pt.sweep.blocks, par, upd);
        }
      }
    return launch_check(c, "gf_batch_run: sweeps");
  };
  for (;;) {
    // check: reunitarise (after the first), measure, copy back
    if (p->reunit_at_check && done > 0) {
      if ((st = tm.begin()) != GF_OK) return st;
      hipLaunchKernelGGL((k_reunitarize_batch<T, NC>), dim3(pt.meas.blocks), dim3(kBlock), 0, c->stream,
                         pt.d_meas, pt.d_meas_map);
      if ((st = tm.end(3, 1)) != GF_OK) return st;
    }
    if ((st = tm.begin()) != GF_OK) return st;
    hipLaunchKernelGGL((k_measure_batch<T, NC>), dim3(pt.meas.blocks), dim3(kBlock), 0, c->stream,
                       pt.d_meas, pt.d_meas_map, b->d_partial);
    hipLaunchKernelGGL((k_finish_batch<T>), dim3(pt.n), dim3(kBlock), 0, c->stream, pt.d_meas, pt.n,
                       pt.meas.blocks, (const double*)b->d_partial, b->d_out, b->d_out + n);
    if ((st = launch_check(c, "gf_batch_run: measure")) != GF_OK) return st;
    if ((st = tm.end(2, 2)) != GF_OK) return st;
    HIP_OR_FAIL(c, hipMemcpyAsync(b->h_out, b->d_out, 2 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    if ((st = tm.flush()) != GF_OK) return st;
    int remaining = 0;
    bool retired = false;
    for (int l = 0; l < n; ++l) {
      if (!b->active[l]) continue;
      const double F = b->h_out[l], th = b->h_out[n + l];
      if (!std::isfinite(F) || !std::isfinite(th))
        return fail(c, GF_ERR_NONFINITE, "gf_batch_run: lattice %d: non-finite F or theta", l);
      ph.F[l] = F;
      ph.theta[l] = th;
      ph.checks[l]++;
      ph.sweeps[l] = done;
      if (th < target) {
        ph.converged[l] = 1;
        b->active[l] = 0;
        retired = true;
      } else if (done >= p->max_sweeps) {
        b->active[l] = 0;
        retired = true;
      } else {
        ++remaining;
      }
    }
    if (!remaining) return GF_OK;
    if (retired) {
      // the stream is idle (synchronised above): rewrite the tables in place
      if ((st = build_tables(b, lo, kSweepKind, pt)) != GF_OK) return st;
      sg.reset();
    }
    const int32_t nsw = std::min(p->check_every, p->max_sweeps - done);
    if (use_graph && nsw == p->check_every && !sg.exec) {
      if (!c->capture) HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
      hipStream_t saved = c->stream;
      c->stream = c->capture;
      hipError_t e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        c->stream = saved;
        return fail(c, GF_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
      }
      st = enqueue(nsw);
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
      sg.n = nsw;
    }
    if ((st = tm.begin()) != GF_OK) return st;
    if (use_graph && sg.exec && nsw == sg.n)
      HIP_OR_FAIL(c, hipGraphLaunch(sg.exec, c->stream));
    else if ((st = enqueue(nsw)) != GF_OK)
      return st;
    if ((st = tm.end(lo ? 0 : 1, 2 * (int64_t)nsw)) != GF_OK) return st;
    done += nsw;
  }
}

template <int NC>
gf_status batch_anneal(gf_batch* b, const gf_fix_params* p, Timer& tm) {
  gf_ctx* c = b->c;
  b->active.assign(b->n, 1);
  PhaseTables<float> pt;
  gf_status st;
  if ((st = build_tables(b, true, kAnnealKind, pt)) != GF_OK) return st;
  for (int32_t k = 0; k < p->sa_steps; ++k) {
    const double T = p->sa_steps > 1
                         ? p->sa_T0 + (p->sa_T1 - p->sa_T0) * (double)k / (double)(p->sa_steps - 1)
                         : p->sa_T0;
    UpdHB<float> hb;
    hb.temp = (float)T;
    hb.k0 = (uint32_t)p->seed;
    hb.k1 = (uint32_t)(p->seed >> 32);
    hb.sweep = (uint32_t)k;
    UpdMicro<float> mc;
    if ((st = tm.begin()) != GF_OK) return st;
    for (int par = 0; par < 2; ++par)
      launch_batch_update<float, NC, UpdHB<float>, true>(c, pt.tps, pt.nt, pt.d_sweep, pt.d_sweep_map, pt.sweep.blocks, par, hb);
    for (int m = 0; m < p->sa_micro; ++m)
      for (int par = 0; par < 2; ++par)
        launch_batch_update<float, NC, UpdMicro<float>, true>(c, pt.tps, pt.nt, pt.d_sweep, pt.d_sweep_map, pt.sweep.blocks, par, mc);
    if ((st = launch_check(c, "gf_batch_run: annealing")) != GF_OK) return st;
    if ((st = tm.end(4, 2 + 2 * (int64_t)p->sa_micro)) != GF_OK) return st;
    if (p->sa_reunit_every > 0 && (k + 1) % p->sa_reunit_every == 0) {
      hipLaunchKernelGGL((k_reunitarize_batch<float, NC>), dim3(pt.meas.blocks), dim3(kBlock), 0, c->stream,
                         pt.d_meas, pt.d_meas_map);
      if ((st = launch_check(c, "gf_batch_run: reunitarise")) != GF_OK) return st;
    }
  }
  return GF_OK;
}

// The batch tuner for one phase: for each lanes count a table over all
// lattices in memory of its own (a captured graph keeps the addresses it was
// given), then the nine variants' blocks of `reps` RED/BLACK pairs captured and
// replayed in turn for five rounds; times[k] = median ms per half-sweep.
template <typename T, int NC, bool TRACK>
gf_status batch_tune_phase(gf_batch* b, bool lo, float times[kVariants]) {
  gf_ctx* c = b->c;
  b->active.assign(b->n, 1);
  struct Dev {
    void* tab = nullptr;
    uint32_t* map = nullptr;
    uint32_t blocks = 0;
  } dev[3];
  auto release = [&]() {
    for (auto& d : dev) {
      if (d.tab) (void)hipFree(d.tab);
      if (d.map) (void)hipFree(d.map);
      d.tab = nullptr;
      d.map = nullptr;
    }
  };
  gf_status st = GF_OK;
  for (int i = 0; i < 3 && st == GF_OK; ++i) {
    const TableSet<T> t = make_table<T>(b, lo, 1 << i);
    dev[i].blocks = t.blocks;
    if (hipMalloc(&dev[i].tab, t.h.size() * sizeof(BatchEntry<T>)) != hipSuccess ||
        hipMalloc((void**)&dev[i].map, t.map.size() * sizeof(uint32_t)) != hipSuccess ||
        hipMemcpy(dev[i].tab, t.h.data(), t.h.size() * sizeof(BatchEntry<T>), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(dev[i].map, t.map.data(), t.map.size() * sizeof(uint32_t), hipMemcpyHostToDevice) !=
            hipSuccess)
      st = fail(c, GF_ERR_HIP, "gf_batch_autotune: launch tables");
  }
  if (st != GF_OK) {
    release();
    return st;
  }
  UpdOR<T> upd;
  upd.omega = (T)1.7;
  auto pair = [&](int tps, int nt) -> gf_status {
    const Dev& d = dev[tps == 1 ? 0 : (tps == 2 ? 1 : 2)];
    for (int par = 0; par < 2; ++par)
      launch_batch_update<T, NC, UpdOR<T>, TRACK>(c, tps, nt, (const BatchEntry<T>*)d.tab, d.map,
                                                  d.blocks, par, upd);
    return launch_check(c, "gf_batch_autotune: sweeps");
  };
  // a block: about 100 ms of work (one pair of the 4-lane cached variant sets it)
  float ms1 = 0;
  if ((st = pair(4, 0)) == GF_OK) {
    (void)hipEventRecord(c->ev[0], c->stream);
    st = pair(4, 0);
    (void)hipEventRecord(c->ev[1], c->stream);
    if (st == GF_OK && (hipEventSynchronize(c->ev[1]) != hipSuccess ||
                        hipEventElapsedTime(&ms1, c->ev[0], c->ev[1]) != hipSuccess))
      st = fail(c, GF_ERR_HIP, "gf_batch_autotune: timing");
  }
  const int reps = std::max(2, std::min(100, (int)std::ceil(100.0 / std::max(ms1, 1e-3f))));
  TuneGraph graphs[kVariants];
  for (int k = 0; k < kVariants && st == GF_OK; ++k)
    st = capture_block(c, [&]() -> gf_status {
      for (int r = 0; r < reps; ++r) {
        gf_status s2 = pair(1 << (k % 3), k / 3);
        if (s2 != GF_OK) return s2;
      }
      return GF_OK;
    }, graphs[k]);
  constexpr int kRounds = 5;
  float t[kVariants][kRounds];
  for (int k = 0; k < kVariants && st == GF_OK; ++k)
    if (hipGraphLaunch(graphs[k].exec, c->stream) != hipSuccess)  // warm-up
      st = fail(c, GF_ERR_HIP, "gf_batch_autotune: replay");
  for (int r = 0; r < kRounds && st == GF_OK; ++r)
    for (int k = 0; k < kVariants && st == GF_OK; ++k) st = time_replay(c, graphs[k], &t[k][r]);
  (void)hipStreamSynchronize(c->stream);
  release();
  if (st != GF_OK) return st;
  for (int k = 0; k < kVariants; ++k) {
    std::sort(t[k], t[k] + kRounds);
    times[k] = t[k][kRounds / 2] / (float)(2 * reps);
  }
  return GF_OK;
}

}  // namespace

gf_status gf_batch_autotune(gf_batch* b, int32_t* tps_out, int32_t* nt_out, float* ms_out) {
  if (!b) return GF_ERR_ARG;
  gf_ctx* c = b->c;
  CHECK_CTX(c);
  const int n = b->n;
  float times[2][kVariants] = {};
  gf_status st = GF_OK;
  // scratch copies of the caller's FP64 fields: the FP64 phase is timed on
  // them, and the FP32 working fields are converted from them
  std::vector<size_t> off(n);
  size_t total = 0;
  for (int l = 0; l < n; ++l) {
    off[l] = total;
    total += (gf_field_bytes(&b->g64[l]) + 255) / 256 * 256;
  }
  void* scratch = nullptr;
  if (hipMalloc(&scratch, total) != hipSuccess)
    return fail(c, GF_ERR_NOMEM, "gf_batch_autotune: scratch copies (%zu bytes)", total);
  std::vector<void*> user = b->U64;
  for (int l = 0; l < n && st == GF_OK; ++l) {
    b->U64[l] = (char*)scratch + off[l];
    if (hipMemcpyAsync(b->U64[l], user[l], gf_field_bytes(&b->g64[l]), hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      st = fail(c, GF_ERR_HIP, "gf_batch_autotune: copy of lattice %d", l);
  }
  // the FP32 phase's fields as gf_batch_run starts them: the input in FP32,
  // g = 1
  for (int l = 0; l < n && st == GF_OK; ++l) {
    st = gf_convert(c, &b->g64[l], b->U64[l], &b->g32[l], (char*)b->arena32 + b->off32[l], 0);
    if (st == GF_OK) {
      hipLaunchKernelGGL((k_fill_unit<float, 6, 1>), dim3(blocks_for(b->lat[l].vp), 2), dim3(kBlock), 0,
                         c->stream, (v2<float>*)((char*)b->arenaG + b->offG[l]), b->lat[l].vp);
      st = launch_check(c, "gf_batch_autotune: init");
    }
  }
  if (st == GF_OK) st = batch_tune_phase<float, 6, true>(b, true, times[0]);
  if (st == GF_OK) {
    if (b->storage == GF_R12)
      st = batch_tune_phase<double, 6, false>(b, false, times[1]);
    else
      st = batch_tune_phase<double, 9, false>(b, false, times[1]);
  }
  (void)hipStreamSynchronize(c->stream);
  b->U64 = user;
  (void)hipFree(scratch);
  if (st != GF_OK) return st;
  for (int ph = 0; ph < 2; ++ph) {
    const bool lo = ph == 0;
    int best = 0;
    for (int k = 1; k < kVariants; ++k)
      if (times[ph][k] < times[ph][best]) best = k;
    b->active.assign(n, 1);
    const gf_geom& g = lo ? b->g32[0] : b->g64[0];
    const int cls = size_class(active_bytes(b, lo));
    ctx_var(c, kSweepKind, g.prec, g.storage, cls).tps = 1 << (best % 3);
    ctx_var(c, kSweepKind, g.prec, g.storage, cls).nt = best / 3;
    if (tps_out) tps_out[ph] = 1 << (best % 3);
    if (nt_out) nt_out[ph] = best / 3;
    if (ms_out)
      for (int k = 0; k < kVariants; ++k) ms_out[9 * ph + k] = times[ph][k];
  }
  return GF_OK;
}

gf_status gf_batch_run(gf_batch* b, const gf_fix_params* p, gf_fix_result* res) {
  if (!b) return GF_ERR_ARG;
  gf_ctx* c = b->c;
  CHECK_CTX(c);
  if (!res) return fail(c, GF_ERR_ARG, "gf_batch_run: NULL results");
  gf_status st = check_params(c, p);
  if (st != GF_OK) return st;
  if (!(p->theta_switch > 0.0)) return fail(c, GF_ERR_ARG, "gf_batch_run: theta_switch must be > 0");
  if (p->or_form != 0) return fail(c, GF_ERR_UNSUPPORTED, "gf_batch_run: or_form must be 0");
  if (p->flags & GF_FLAG_FREEZE_TIMESLICES)
    return fail(c, GF_ERR_UNSUPPORTED, "gf_batch_run: GF_FLAG_FREEZE_TIMESLICES (batches are Landau)");
  const int n = b->n;
  for (int l = 0; l < n; ++l) init_result(&res[l]);
  const auto t0 = std::chrono::steady_clock::now();
  Timer tm{c, (p->flags & GF_FLAG_TIMING) != 0, res[0].kernel_ms, res[0].kernel_launches};
  // FP64 inputs -> FP32 working fields, g = 1
  if ((st = tm.begin()) != GF_OK) return st;
  for (int l = 0; l < n && st == GF_OK; ++l) {
    st = gf_convert(c, &b->g64[l], b->U64[l], &b->g32[l], (char*)b->arena32 + b->off32[l], 0);
    if (st == GF_OK) {
      hipLaunchKernelGGL((k_fill_unit<float, 6, 1>), dim3(blocks_for(b->lat[l].vp), 2), dim3(kBlock), 0,
                         c->stream, (v2<float>*)((char*)b->arenaG + b->offG[l]), b->lat[l].vp);
      st = launch_check(c, "gf_batch_run: init");
    }
  }
  if (st == GF_OK) st = tm.end(3, 2 * n);
  if (st == GF_OK && p->sa_steps > 0) st = batch_anneal<6>(b, p, tm);
  BatchPhase lo, hi;
  if (st == GF_OK) st = batch_phase<float, 6>(b, p, true, p->theta_switch, tm, lo);
  if (st == GF_OK) {
    if ((st = tm.begin()) == GF_OK) {
      for (int l = 0; l < n && st == GF_OK; ++l) {
        const Lat& L = b->lat[l];
        const v2<float>* G = (const v2<float>*)((char*)b->arenaG + b->offG[l]);
        if (b->storage == GF_R12)
          hipLaunchKernelGGL((k_apply_gauge<double, 6, float>), dim3(blocks_for(L.vh), 2), dim3(kBlock), 0,
                             c->stream, (v2<double>*)b->U64[l], G, L);
        else
          hipLaunchKernelGGL((k_apply_gauge<double, 9, float>), dim3(blocks_for(L.vh), 2), dim3(kBlock), 0,
                             c->stream, (v2<double>*)b->U64[l], G, L);
        st = launch_check(c, "gf_batch_run: apply g");
      }
      if (st == GF_OK) st = tm.end(3, n);
    }
  }
  if (st == GF_OK)
    st = b->storage == GF_R12 ? batch_phase<double, 6>(b, p, false, p->theta_target, tm, hi)
                              : batch_phase<double, 9>(b, p, false, p->theta_target, tm, hi);
  if (st == GF_OK) st = tm.flush();
  const double wall =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int l = 0; l < n; ++l) {
    gf_fix_result& r = res[l];
    r.sa_steps = p->sa_steps;
    if (!lo.sweeps.empty()) {
      r.sweeps_lo = lo.sweeps[l];
      r.theta_at_switch = lo.theta[l];
      r.checks = lo.checks[l];
      r.F = lo.F[l];
      r.theta = lo.theta[l];
    }
    if (!hi.sweeps.empty()) {
      r.sweeps = r.sweeps_lo + hi.sweeps[l];
      r.checks += hi.checks[l];
      r.F = hi.F[l];
      r.theta = hi.theta[l];
      r.status = hi.converged[l] ? GF_OK : GF_NOT_CONVERGED;
    } else {
      r.sweeps = r.sweeps_lo;
      r.status = st != GF_OK ? st : GF_NOT_CONVERGED;
    }
    r.wall_ms = wall;
  }
  if (st != GF_OK) return st;
  for (int l = 0; l < n; ++l)
    if (res[l].status != GF_OK) return GF_NOT_CONVERGED;
  return GF_OK;
}
