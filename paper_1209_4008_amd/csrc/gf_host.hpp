// gf_host.hpp -- host-side internals shared by the translation units of
// libgf: the context, argument validation, geometry, the error channel and the
// templated kernel dispatch over (precision, storage, gauge, lanes per site,
// nontemporal mode). The C ABI is declared in include/gf.h; each entry point
// lives in one translation unit, so that the kernels it instantiates are
// compiled there and the units build in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/gf.h"
#include "gf_kernels.hpp"

using namespace gf;

struct gf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char err[512] = {0};
  double* partial = nullptr;  // per-block reduction partials
  size_t partial_cap = 0;     // doubles
  double* dev_out = nullptr;  // driver F/theta outputs (2 x out_cap doubles)
  double* host_out = nullptr; // pinned copy of dev_out
  size_t out_cap = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // sweep-kernel variants set or tuned on this context, [kind][fp64][r18][size
  // class]: kind 0 the overrelaxation sweeps (every form, stochastic
  // relaxation, MAG), 1 the annealing updates (heatbath, microcanonical); size
  // class 0 fields of at most 2 GiB, 1 larger ones. tps = lanes per site (0:
  // built-in), nt = nontemporal mode (-1: built-in).
  struct Variant {
    int tps = 0;
    int nt = -1;
  } var[2][2][2][2];
  void* gbuf = nullptr;  // gauge-transformation field of the mixed driver
  size_t gbuf_cap = 0;   // bytes
  hipStream_t capture = nullptr;  // private stream for hipGraph capture
  std::vector<hipEvent_t> pool;   // driver timing events, pairs (start, end)
  // Coulomb drivers with GF_FLAG_FREEZE_TIMESLICES: one byte per timeslice,
  // 0 = frozen; `tmask` is what the sweep launches pass (NULL outside such a
  // driver call)
  uint8_t* dev_tmask = nullptr;
  uint8_t* host_tmask = nullptr;  // pinned
  size_t tmask_cap = 0;
  const uint8_t* tmask = nullptr;
  // the drivers' unitarity monitor (GF_FLAG_MONITOR): 1 double each
  double* dev_mon = nullptr;
  double* host_mon = nullptr;  // pinned
};

// message of the last failed call made without a context (gf_create)
extern char g_create_err[512];

static inline gf_status fail(gf_ctx* c, gf_status st, const char* fmt, ...) {
  char* dst = c ? c->err : g_create_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return st;
}

#define HIP_OR_FAIL(ctx, expr)                                                       \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail((ctx), GF_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                               \
  } while (0)
static inline gf_status launch_check(gf_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, GF_ERR_HIP, "%s: launch failed: %s", what, hipGetErrorString(e));
  return GF_OK;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
static inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  uint32_t l = 0;
  while (((uint64_t)1 << l) < d) ++l;
  f.d = d;
  f.shift = 32 + l;
  // m = ceil(2^(32+l) / d)
  const unsigned __int128 num = (unsigned __int128)1 << (32 + l);
  f.m = (uint64_t)((num + d - 1) / d);
  return f;
}

static inline uint32_t host_fdiv(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((unsigned __int128)n * f.m) >> f.shift);
}

static inline int geom_ok(const gf_geom* g) {
  if (!g) return 0;
  const int32_t e[4] = {g->nt, g->nz, g->ny, g->nx};
  for (int k = 0; k < 4; ++k)
    if (e[k] < 2 || (e[k] & 1) || e[k] > 65536) return 0;
  if (g->prec != GF_FP32 && g->prec != GF_FP64) return 0;
  if (g->storage != GF_R12 && g->storage != GF_R18) return 0;
  const uint64_t V = (uint64_t)g->nt * g->nz * g->ny * g->nx;
  if (V > ((uint64_t)1 << 30)) return 0;
  return 1;
}

static inline Lat make_lat(const gf_geom* g) {
  Lat L;
  L.nt = g->nt;
  L.nz = g->nz;
  L.ny = g->ny;
  L.nx = g->nx;
  L.hx = g->nx / 2;
  L.vh = (uint32_t)((uint64_t)g->nt * g->nz * g->ny * g->nx / 2);
  L.vp = (uint32_t)padded_half(L.vh);
  L.sy = L.hx;
  L.sz = L.ny * L.hx;
  L.st = L.nz * L.ny * L.hx;
  L.div_hx = make_fastdiv(L.hx);
  L.div_ny = make_fastdiv(L.ny);
  L.div_nz = make_fastdiv(L.nz);
  return L;
}

static inline int same_extents(const gf_geom* a, const gf_geom* b) {
  return a->nt == b->nt && a->nz == b->nz && a->ny == b->ny && a->nx == b->nx;
}

// ---------------------------------------------------------------------------
// dispatch helpers
// ---------------------------------------------------------------------------
template <class F>
static inline void with_type(const gf_geom* g, F&& f) {
  if (g->prec == GF_FP32) {
    if (g->storage == GF_R12)
      f.template operator()<float, 6>();
    else
      f.template operator()<float, 9>();
  } else {
    if (g->storage == GF_R12)
      f.template operator()<double, 6>();
    else
      f.template operator()<double, 9>();
  }
}

static inline unsigned blocks_for(uint64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

static inline gf_status ensure_partial(gf_ctx* c, size_t n_doubles) {
  if (n_doubles <= c->partial_cap) return GF_OK;
  if (c->partial) HIP_OR_FAIL(c, hipFree(c->partial));
  c->partial = nullptr;
  c->partial_cap = 0;
  HIP_OR_FAIL(c, hipMalloc(&c->partial, n_doubles * sizeof(double)));
  c->partial_cap = n_doubles;
  return GF_OK;
}

static inline gf_status ensure_tmask(gf_ctx* c, size_t n) {
  if (n <= c->tmask_cap) return GF_OK;
  if (c->dev_tmask) HIP_OR_FAIL(c, hipFree(c->dev_tmask));
  if (c->host_tmask) HIP_OR_FAIL(c, hipHostFree(c->host_tmask));
  c->dev_tmask = nullptr;
  c->host_tmask = nullptr;
  c->tmask_cap = 0;
  HIP_OR_FAIL(c, hipMalloc(&c->dev_tmask, n));
  HIP_OR_FAIL(c, hipHostMalloc(&c->host_tmask, n, hipHostMallocDefault));
  c->tmask_cap = n;
  return GF_OK;
}

static inline gf_status ensure_mon(gf_ctx* c) {
  if (c->dev_mon) return GF_OK;
  HIP_OR_FAIL(c, hipMalloc(&c->dev_mon, sizeof(double)));
  if (hipHostMalloc(&c->host_mon, sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(c->dev_mon);
    c->dev_mon = nullptr;
    return fail(c, GF_ERR_HIP, "hipHostMalloc of the monitor output failed");
  }
  return GF_OK;
}

static inline gf_status ensure_out(gf_ctx* c, size_t n) {
  if (n <= c->out_cap) return GF_OK;
  if (c->dev_out) HIP_OR_FAIL(c, hipFree(c->dev_out));
  if (c->host_out) HIP_OR_FAIL(c, hipHostFree(c->host_out));
  c->dev_out = nullptr;
  c->host_out = nullptr;
  c->out_cap = 0;
  HIP_OR_FAIL(c, hipMalloc(&c->dev_out, 2 * n * sizeof(double)));
  HIP_OR_FAIL(c, hipHostMalloc(&c->host_out, 2 * n * sizeof(double), hipHostMallocDefault));
  c->out_cap = n;
  return GF_OK;
}
// every entry point starts by clearing a stale per-thread HIP error (left by
// some earlier, unrelated runtime call), so that launch_check reports the
// entry point's own launches
#define CHECK_CTX(c)                                                    \
  do {                                                                  \
    if (!(c)) return GF_ERR_ARG;                                        \
    (void)hipGetLastError();                                            \
    if (hipSetDevice((c)->device) != hipSuccess)                        \
      return fail((c), GF_ERR_DEVICE, "hipSetDevice(%d) failed", (c)->device); \
  } while (0)

#define CHECK_GEOM(c, g, what) \
  if (!geom_ok(g)) return fail((c), GF_ERR_ARG, "%s: invalid geometry", what)
constexpr int kSweepKind = 0, kAnnealKind = 1;
// variants timed by the autotuner: lanes per site 1, 2, 4 x nontemporal mode
// kNTNone, kNTAll, kNTStores, index 3 * mode + log2(lanes)
constexpr int kVariants = 9;
// Built-in nontemporal mode: ordinary (cached) accesses, with which the
// alternating sweep direction lets the Infinity Cache serve the start of
// every half-sweep. Fields many times larger than the 256 MB cache gain
// nothing from it, and over several GB streamed accesses run faster (FP64
// 12-real, 4 lanes: 56^4, 3.8 GB, 5.2 against 4.9 TB/s; 64^4, 6.4 GB, 5.5
// against 5.3; 72^4, 10.3 GB, 5.1 against 4.5; at 48^4, 2 GB, the modes are
// within 2%), so above 2 GiB the built-in mode streams loads and stores.
constexpr size_t kStreamBytes = (size_t)2 << 30;
static inline int default_nt_bytes(size_t bytes) { return bytes > kStreamBytes ? kNTAll : kNTNone; }
static inline int default_nt(const gf_geom* g) { return default_nt_bytes(gf_field_bytes(g)); }
// Built-in lanes per site, for launches over `bytes` of fields. FP64: 4 lanes
// (three waves per SIMD) with the cached accesses of fields up to 2 GiB; one
// lane (all 8 links of a site in its registers, one wave per SIMD) with the
// streamed accesses above, where it sweeps fastest: the 192-lattice batch
// (10.8 GB) FP64 half-sweep 3.55 ms with 1 lane against 3.86 ms with 4 and
// 4.08 ms with 2. FP32 overrelaxation 2. The FP32 annealing updates run 1
// lane: the heatbath's draws and trials then cost a lane no more than with
// 2 lanes, and at 32^3 x 64 (tracked, 12 reals) 1 lane took 143.4 / 145.6 /
// 171.8 us per half-sweep at T = 0.05 / 0.5 / 1.45 against 155.4 / 157.3 /
// 169.4 with 2 (microcanonical 143.7 against 144.8).
static inline int default_tps_bytes(const gf_geom* g, int kind, size_t bytes) {
  if (g->prec == GF_FP64) return (kind == kSweepKind && bytes > kStreamBytes) ? 1 : 4;
  return kind == kAnnealKind ? 1 : 2;
}

// the stores-only nontemporal mode is instantiated for the overrelaxation
// sweeps (all forms of g^omega and stochastic relaxation: the same
// bandwidth-bound sweep the autotuner times); the annealing updates run it
// as kNTAll
template <class Upd>
struct HasStoreMode {
  static constexpr bool value = false;
};
template <typename T>
struct HasStoreMode<UpdOR<T>> {
  static constexpr bool value = true;
};
template <typename T>
struct HasStoreMode<UpdORForm<T>> {
  static constexpr bool value = true;
};
template <typename T>
struct HasStoreMode<UpdSR<T>> {
  static constexpr bool value = true;
};
template <class Upd>
static inline int nt_mode(int nt) {
  if (nt == kNTStores && !HasStoreMode<Upd>::value) return kNTAll;
  return nt;
}

template <typename T, int NC, int GAUGE, class Upd, int NT>
static inline void launch_update_v(gf_ctx* c, int tps, void* U, const Lat& L, int parity, const Upd& upd) {
  const uint8_t* tm = GAUGE == kCoulomb ? c->tmask : nullptr;
  const uint64_t n = (uint64_t)L.vh * (uint64_t)tps;
  const dim3 grid(blocks_for(n));
  switch (tps) {
    case 1:
      hipLaunchKernelGGL((k_update_half<T, NC, GAUGE, Upd, 1, NT>), grid, dim3(kBlock), 0, c->stream,
                         (v2<T>*)U, L, parity, upd, (v2<T>*)nullptr, tm);
      break;
    case 2:
      hipLaunchKernelGGL((k_update_half<T, NC, GAUGE, Upd, 2, NT>), grid, dim3(kBlock), 0, c->stream,
                         (v2<T>*)U, L, parity, upd, (v2<T>*)nullptr, tm);
      break;
    default:
      hipLaunchKernelGGL((k_update_half<T, NC, GAUGE, Upd, 4, NT>), grid, dim3(kBlock), 0, c->stream,
                         (v2<T>*)U, L, parity, upd, (v2<T>*)nullptr, tm);
      break;
  }
}

// the MAG site update takes the overrelaxation policies only
template <class Upd>
struct MagCapable {
  static constexpr bool value = false;
};
template <typename T>
struct MagCapable<UpdOR<T>> {
  static constexpr bool value = true;
};
template <typename T>
struct MagCapable<UpdORForm<T>> {
  static constexpr bool value = true;
};

template <typename T, int NC, class Upd, int NT, bool TRACK>
static inline void launch_mag_v(gf_ctx* c, int tps, void* U, void* Gx, const Lat& L, int parity,
                         const Upd& upd) {
  const dim3 grid(blocks_for((uint64_t)L.vh * (uint64_t)tps));
  switch (tps) {
    case 1:
      hipLaunchKernelGGL((k_mag_half<T, NC, Upd, 1, NT, TRACK>), grid, dim3(kBlock), 0, c->stream,
                         (v2<T>*)U, L, parity, upd, (v2<T>*)Gx);
      break;
    case 2:
      hipLaunchKernelGGL((k_mag_half<T, NC, Upd, 2, NT, TRACK>), grid, dim3(kBlock), 0, c->stream,
                         (v2<T>*)U, L, parity, upd, (v2<T>*)Gx);
      break;
    default:
      hipLaunchKernelGGL((k_mag_half<T, NC, Upd, 4, NT, TRACK>), grid, dim3(kBlock), 0, c->stream,
                         (v2<T>*)U, L, parity, upd, (v2<T>*)Gx);
      break;
  }
}

template <typename T, int NC, int GAUGE, class Upd>
static inline void launch_update_tps(gf_ctx* c, int tps, int nt, void* U, const Lat& L, int parity,
                              const Upd& upd) {
  if constexpr (GAUGE == kMAG) {
    if constexpr (MagCapable<Upd>::value) {
      const int mode = nt_mode<Upd>(nt);
      if (mode == kNTAll)
        launch_mag_v<T, NC, Upd, kNTAll, false>(c, tps, U, nullptr, L, parity, upd);
      else if (mode == kNTStores) {
        if constexpr (HasStoreMode<Upd>::value)
          launch_mag_v<T, NC, Upd, kNTStores, false>(c, tps, U, nullptr, L, parity, upd);
      } else
        launch_mag_v<T, NC, Upd, kNTNone, false>(c, tps, U, nullptr, L, parity, upd);
    }
    return;
  }
  const int mode = nt_mode<Upd>(nt);
  if (mode == kNTAll) {
    launch_update_v<T, NC, GAUGE, Upd, kNTAll>(c, tps, U, L, parity, upd);
  } else if (mode == kNTStores) {
    if constexpr (HasStoreMode<Upd>::value)
      launch_update_v<T, NC, GAUGE, Upd, kNTStores>(c, tps, U, L, parity, upd);
  } else {
    launch_update_v<T, NC, GAUGE, Upd, kNTNone>(c, tps, U, L, parity, upd);
  }
}

// FP32 half-sweep (any update) that also accumulates g(x) <- Gtot g(x) into Gx
template <int NC, int GAUGE, int NT, class Upd>
static inline void launch_tracked_v(gf_ctx* c, int tps, void* U, void* Gx, const Lat& L, int parity,
                             const Upd& upd) {
  const uint8_t* tm = GAUGE == kCoulomb ? c->tmask : nullptr;
  const dim3 grid(blocks_for((uint64_t)L.vh * (uint64_t)tps));
  switch (tps) {
    case 1:
      hipLaunchKernelGGL((k_update_half<float, NC, GAUGE, Upd, 1, NT, true>), grid, dim3(kBlock), 0,
                         c->stream, (v2<float>*)U, L, parity, upd, (v2<float>*)Gx, tm);
      break;
    case 2:
      hipLaunchKernelGGL((k_update_half<float, NC, GAUGE, Upd, 2, NT, true>), grid, dim3(kBlock), 0,
                         c->stream, (v2<float>*)U, L, parity, upd, (v2<float>*)Gx, tm);
      break;
    default:
      hipLaunchKernelGGL((k_update_half<float, NC, GAUGE, Upd, 4, NT, true>), grid, dim3(kBlock), 0,
                         c->stream, (v2<float>*)U, L, parity, upd, (v2<float>*)Gx, tm);
      break;
  }
}

static inline int size_class(size_t bytes) { return bytes > kStreamBytes ? 1 : 0; }
static inline gf_ctx::Variant& ctx_var(gf_ctx* c, int kind, int prec, int storage, int cls) {
  return c->var[kind][prec == GF_FP64][storage == GF_R18][cls];
}
static inline const gf_ctx::Variant& ctx_var(const gf_ctx* c, int kind, const gf_geom* g,
                                             size_t bytes) {
  return c->var[kind][g->prec == GF_FP64][g->storage == GF_R18][size_class(bytes)];
}
// the variant of a launch over fields of `bytes` in all (batches: the active
// lattices' fields), of geometry g's precision and storage
static inline int ctx_tps_bytes(const gf_ctx* c, const gf_geom* g, int kind, size_t bytes) {
  const int t = ctx_var(c, kind, g, bytes).tps;
  return t > 0 ? t : default_tps_bytes(g, kind, bytes);
}
static inline int ctx_nt_bytes(const gf_ctx* c, const gf_geom* g, int kind, size_t bytes) {
  const int t = ctx_var(c, kind, g, bytes).nt;
  return t >= 0 ? t : default_nt_bytes(bytes);
}
static inline int ctx_tps(const gf_ctx* c, const gf_geom* g, int kind = kSweepKind) {
  return ctx_tps_bytes(c, g, kind, gf_field_bytes(g));
}
static inline int ctx_nt(const gf_ctx* c, const gf_geom* g, int kind = kSweepKind) {
  return ctx_nt_bytes(c, g, kind, gf_field_bytes(g));
}
// which variant table an update policy uses
template <class Upd>
struct UpdKind {
  static constexpr int value = kSweepKind;
};
template <typename T>
struct UpdKind<UpdHB<T>> {
  static constexpr int value = kAnnealKind;
};
template <typename T>
struct UpdKind<UpdMicro<T>> {
  static constexpr int value = kAnnealKind;
};

template <class UpdF>
static inline gf_status launch_update(gf_ctx* c, void* U, const gf_geom* g, int32_t gauge,
                               int32_t parity, UpdF make_upd, const char* what) {
  using UpdD = decltype(make_upd.template operator()<double>());
  if (gauge == GF_MAG && !MagCapable<UpdD>::value)
    return fail(c, GF_ERR_UNSUPPORTED, "%s: not available for GF_MAG", what);
  const Lat L = make_lat(g);
  const int kind = UpdKind<UpdD>::value;
  const int tps = ctx_tps(c, g, kind), nt = ctx_nt(c, g, kind);
  with_type(g, [&]<typename T, int NC>() {
    auto upd = make_upd.template operator()<T>();
    if (gauge == GF_LANDAU)
      launch_update_tps<T, NC, kLandau>(c, tps, nt, U, L, (int)parity, upd);
    else if (gauge == GF_COULOMB)
      launch_update_tps<T, NC, kCoulomb>(c, tps, nt, U, L, (int)parity, upd);
    else
      launch_update_tps<T, NC, kMAG>(c, tps, nt, U, L, (int)parity, upd);
  });
  return launch_check(c, what);
}

#define CHECK_GAUGE_PARITY(c, gauge, parity, what)                                    \
  if ((gauge) != GF_LANDAU && (gauge) != GF_COULOMB && (gauge) != GF_MAG)             \
    return fail((c), GF_ERR_ARG, "%s: gauge must be GF_LANDAU, GF_COULOMB or GF_MAG", what); \
  if ((parity) != 0 && (parity) != 1) return fail((c), GF_ERR_ARG, "%s: parity must be 0 or 1", what)
// the annealing and stochastic-relaxation updates are defined for the linear
// functionals of Landau and Coulomb gauge only
#define REJECT_MAG(c, gauge, what) \
  if ((gauge) == GF_MAG) return fail((c), GF_ERR_UNSUPPORTED, "%s: not available for GF_MAG", what)
// FP32 half-sweep with g tracking (mixed-precision driver)
template <class Upd>
static inline gf_status update_tracked(gf_ctx* c, void* U, void* Gx, const gf_geom* g, int32_t gauge,
                                int32_t parity, const Upd& upd, const char* what) {
  if (gauge == GF_MAG && !MagCapable<Upd>::value)
    return fail(c, GF_ERR_UNSUPPORTED, "%s: not available for GF_MAG", what);
  const Lat L = make_lat(g);
  const int kind = UpdKind<Upd>::value;
  const int tps = ctx_tps(c, g, kind), nt = ctx_nt(c, g, kind);
  const int mode = nt_mode<Upd>(nt);
  auto go_gauge = [&]<int NC, int GAUGE>() {
    if (mode == kNTAll) {
      launch_tracked_v<NC, GAUGE, kNTAll>(c, tps, U, Gx, L, parity, upd);
    } else if (mode == kNTStores) {
      if constexpr (HasStoreMode<Upd>::value)
        launch_tracked_v<NC, GAUGE, kNTStores>(c, tps, U, Gx, L, parity, upd);
    } else {
      launch_tracked_v<NC, GAUGE, kNTNone>(c, tps, U, Gx, L, parity, upd);
    }
  };
  auto go = [&]<int NC>() {
    if (gauge == GF_LANDAU) {
      go_gauge.template operator()<NC, kLandau>();
    } else if (gauge == GF_MAG) {
      if constexpr (MagCapable<Upd>::value) {
        if (mode == kNTAll) {
          launch_mag_v<float, NC, Upd, kNTAll, true>(c, tps, U, Gx, L, parity, upd);
        } else if (mode == kNTStores) {
          if constexpr (HasStoreMode<Upd>::value)
            launch_mag_v<float, NC, Upd, kNTStores, true>(c, tps, U, Gx, L, parity, upd);
        } else {
          launch_mag_v<float, NC, Upd, kNTNone, true>(c, tps, U, Gx, L, parity, upd);
        }
      }
    } else {
      go_gauge.template operator()<NC, kCoulomb>();
    }
  };
  if (g->storage == GF_R12)
    go.template operator()<6>();
  else
    go.template operator()<9>();
  return launch_check(c, what);
}

// ---------------------------------------------------------------------------
// tuner timing (gf_core.hip: single fields, gf_batch.hip: batches)
// ---------------------------------------------------------------------------
// One captured block of timing work per variant, replayed from a hipGraph as
// the drivers replay their sweep blocks.
struct TuneGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~TuneGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// capture `enqueue` (which launches on c->stream) into g on the context's
// capture stream
template <class F>
inline gf_status capture_block(gf_ctx* c, F&& enqueue, TuneGraph& g) {
  if (!c->capture) HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
  hipStream_t saved = c->stream;
  c->stream = c->capture;
  hipError_t e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    c->stream = saved;
    return fail(c, GF_ERR_HIP, "autotune: hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  gf_status st = enqueue();
  e = hipStreamEndCapture(c->capture, &g.graph);
  c->stream = saved;
  if (st != GF_OK) return st;
  if (e != hipSuccess) return fail(c, GF_ERR_HIP, "autotune: hipStreamEndCapture: %s", hipGetErrorString(e));
  HIP_OR_FAIL(c, hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
  return GF_OK;
}

// time one replay of g on the context stream (ms)
inline gf_status time_replay(gf_ctx* c, const TuneGraph& g, float* ms) {
  HIP_OR_FAIL(c, hipEventRecord(c->ev[0], c->stream));
  HIP_OR_FAIL(c, hipGraphLaunch(g.exec, c->stream));
  HIP_OR_FAIL(c, hipEventRecord(c->ev[1], c->stream));
  HIP_OR_FAIL(c, hipEventSynchronize(c->ev[1]));
  HIP_OR_FAIL(c, hipEventElapsedTime(ms, c->ev[0], c->ev[1]));
  return GF_OK;
}

// ---------------------------------------------------------------------------
// internal functions shared between the units (C++ linkage)
// ---------------------------------------------------------------------------
// gf_core.hip: F and theta of a field into F, th (either may be NULL)
gf_status measure_impl(gf_ctx* c, const void* U, const gf_geom* g, int32_t gauge, double* F,
                       double* th);
// gf_tracked_or.hip: FP32 overrelaxation half-sweeps that also accumulate the
// site transformation into the gauge-transformation field Gx
gf_status sweep_tracked(gf_ctx* c, void* U, void* Gx, const gf_geom* g, int32_t gauge,
                        int32_t parity, double omega);
gf_status sweep_form_tracked(gf_ctx* c, void* U, void* Gx, const gf_geom* g, int32_t gauge,
                             int32_t parity, double omega, int32_t form);
// gf_tracked_anneal.hip: the same for stochastic relaxation and annealing
gf_status sweep_sr_tracked(gf_ctx* c, void* U, void* Gx, const gf_geom* g, int32_t gauge,
                           int32_t parity, double omega, double prob, uint64_t seed,
                           uint64_t sweep);
gf_status anneal_step_tracked(gf_ctx* c, void* U, void* Gx, const gf_geom* g, int32_t gauge,
                              double T, uint64_t seed, uint64_t sweep, int32_t n_micro);
// gf_monitor.hip: the unitarity deviation of a field into out (device, 1 double)
gf_status unitarity_launch(gf_ctx* c, const void* U, const gf_geom* g, double* out);

// validation shared by the tracked entry points
#define CHECK_TRACKED(c, U, G, g, what)                                                  \
  do {                                                                                   \
    if (!(U) || !(G)) return fail((c), GF_ERR_ARG, "%s: NULL pointer", what);            \
    if ((g)->prec != GF_FP32)                                                            \
      return fail((c), GF_ERR_UNSUPPORTED, "%s: FP32 fields only", what);                \
    const char *a_ = (const char*)(U), *b_ = (const char*)(G);                           \
    if (a_ < b_ + gf_gauge_bytes(g) && b_ < a_ + gf_field_bytes(g))                      \
      return fail((c), GF_ERR_ARG, "%s: field and gauge field overlap", what);           \
  } while (0)
