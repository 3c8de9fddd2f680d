// gf_core.hip -- libgf context, layout conversion, reductions, tuning and
// bandwidth probes.
#include "gf_host.hpp"

#include <mutex>

char g_create_err[512] = "no error";

// ---------------------------------------------------------------------------
// C ABI (C linkage comes from the declarations in gf.h)
// ---------------------------------------------------------------------------

const char* gf_version(void) { return "libgf 0.1 (gfx950)"; }

gf_status gf_check_geom(const gf_geom* geom) { return geom_ok(geom) ? GF_OK : GF_ERR_ARG; }

size_t gf_field_bytes(const gf_geom* geom) {
  if (!geom_ok(geom)) return 0;
  const uint64_t V = (uint64_t)geom->nt * geom->nz * geom->ny * geom->nx;
  return (size_t)(8 * padded_half(V / 2) * (uint64_t)geom->storage * (uint64_t)geom->prec);
}

// The device index arithmetic (site_of, back_h, fwd_h) run on the host for
// every site of a set of lattices, against the canonical definition
// s = ((t*nz + z)*ny + y)*nx + x, parity (t+x+y+z) mod 2, h = s >> 1.
static int selftest_lattice(int nt, int nz, int ny, int nx) {
  gf_geom g = {nt, nz, ny, nx, GF_FP64, GF_R18};
  const Lat L = make_lat(&g);
  auto canon = [&](int64_t t, int64_t z, int64_t y, int64_t x) {
    return ((t * nz + z) * ny + y) * nx + x;
  };
  for (int p = 0; p < 2; ++p)
    for (uint32_t h = 0; h < L.vh; ++h) {
      const Site S = site_of(L, h, p);
      if (S.t >= (uint32_t)nt || S.z >= (uint32_t)nz || S.y >= (uint32_t)ny || S.x >= (uint32_t)nx)
        return 0;
      const int64_t s = canon(S.t, S.z, S.y, S.x);
      if ((s >> 1) != h || (int)((S.t + S.z + S.y + S.x) & 1) != p || S.xodd != (S.x & 1)) return 0;
      const int64_t c[4] = {S.t, S.x, S.y, S.z};
      const int64_t e[4] = {nt, nx, ny, nz};
      for (int mu = 0; mu < 4; ++mu) {
        int64_t b[4] = {c[0], c[1], c[2], c[3]}, f[4] = {c[0], c[1], c[2], c[3]};
        b[mu] = (b[mu] - 1 + e[mu]) % e[mu];
        f[mu] = (f[mu] + 1) % e[mu];
        const uint32_t hb = back_h(L, h, S, mu), hf = fwd_h(L, h, S, mu);
        if (hb >= L.vh || hf >= L.vh) return 0;
        if ((uint64_t)(canon(b[0], b[3], b[2], b[1]) >> 1) != hb) return 0;
        if ((uint64_t)(canon(f[0], f[3], f[2], f[1]) >> 1) != hf) return 0;
      }
    }
  // the tiled element offsets of every (parity, direction, component, site)
  // are distinct and lie inside the field of 8 * NC * vp elements; the same
  // for the one-matrix-per-site fields (2 * 6 * vp elements)
  if (L.vp % kTile != 0 || L.vp < L.vh || L.vp - L.vh >= kTile) return 0;
  {
    std::vector<unsigned char> seen((size_t)2 * 6 * L.vp, 0);
    for (int pp = 0; pp < 2; ++pp)
      for (uint32_t h = 0; h < L.vh; ++h)
        for (int cc = 0; cc < 6; ++cc) {
          const size_t e = link_offset<6, 1>(L.vp, pp, 0, h) + (size_t)cc * kTile;
          if (e >= seen.size() || seen[e]) return 0;
          seen[e] = 1;
        }
  }
  for (int NC : {6, 9}) {
    std::vector<unsigned char> seen((size_t)8 * NC * L.vp, 0);
    for (uint32_t pm = 0; pm < 8; ++pm)
      for (uint32_t h = 0; h < L.vh; ++h) {
        const int pp = (int)(pm >> 2), mu = (int)(pm & 3);
        const size_t base = NC == 6 ? link_offset<6>(L.vp, pp, mu, h) : link_offset<9>(L.vp, pp, mu, h);
        for (int cc = 0; cc < NC; ++cc) {
          const size_t e = base + (size_t)cc * kTile;
          if (e >= seen.size() || seen[e]) return 0;
          seen[e] = 1;
        }
      }
  }
  return 1;
}

gf_status gf_selftest_host(void) {
  // exact division for the divisors the geometry can produce
  for (uint32_t d = 1; d <= 4096; d = d < 64 ? d + 1 : d + 37) {
    const FastDiv f = make_fastdiv(d);
    const uint32_t probes[] = {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 1000003u, 0x7ffffffeu,
                               0x7fffffffu, 123456789u};
    for (uint32_t n : probes)
      if (host_fdiv(n, f) != n / d || fdiv(n, f) != n / d) return GF_ERR_UNSUPPORTED;
    for (uint32_t n = 0; n < 5000; ++n)
      if (fdiv(n * 7919u, f) != (n * 7919u) / d) return GF_ERR_UNSUPPORTED;
  }
  const int shapes[][4] = {{2, 2, 2, 2},     {4, 4, 4, 4},    {6, 4, 2, 10},  {4, 6, 8, 10},
                           {8, 2, 6, 4},     {2, 12, 2, 14},  {10, 6, 4, 2},  {24, 12, 12, 12},
                           {2, 2, 2, 65536}, {2, 2, 32768, 4}, {2, 16384, 2, 6}, {32768, 2, 2, 2}};
  for (const auto& d : shapes)
    if (!selftest_lattice(d[0], d[1], d[2], d[3])) return GF_ERR_UNSUPPORTED;
  return GF_OK;
}

const char* gf_last_error(const gf_ctx* ctx) { return ctx ? ctx->err : g_create_err; }

static gf_status scratch_setup(int device);  // the static measurement scratch, below

gf_status gf_create(int device, void* hip_stream, gf_ctx** out) {
  if (!out) return fail(nullptr, GF_ERR_ARG, "gf_create: out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
    return fail(nullptr, GF_ERR_DEVICE, "gf_create: no GPU device available");
  if (device < 0 || device >= n)
    return fail(nullptr, GF_ERR_ARG, "gf_create: device %d out of range (%d devices)", device, n);
  if (hipSetDevice(device) != hipSuccess)
    return fail(nullptr, GF_ERR_DEVICE, "gf_create: hipSetDevice(%d) failed", device);
  {
    const gf_status st = scratch_setup(device);
    if (st != GF_OK) return st;
  }
  gf_ctx* c = new gf_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess) {
    delete c;
    return fail(nullptr, GF_ERR_HIP, "gf_create: hipEventCreate failed");
  }
  snprintf(c->err, sizeof c->err, "no error");
  *out = c;
  return GF_OK;
}

gf_status gf_destroy(gf_ctx* c) {
  if (!c) return GF_ERR_ARG;
  (void)hipSetDevice(c->device);
  if (c->partial) (void)hipFree(c->partial);
  if (c->dev_out) (void)hipFree(c->dev_out);
  if (c->host_out) (void)hipHostFree(c->host_out);
  if (c->gbuf) (void)hipFree(c->gbuf);
  if (c->dev_tmask) (void)hipFree(c->dev_tmask);
  if (c->host_tmask) (void)hipHostFree(c->host_tmask);
  if (c->dev_mon) (void)hipFree(c->dev_mon);
  if (c->host_mon) (void)hipHostFree(c->host_mon);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  for (auto& e : c->pool) (void)hipEventDestroy(e);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return GF_OK;
}

gf_status gf_pack(gf_ctx* c, const gf_geom* g, const double* src, void* dst) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_pack");
  if (!src || !dst) return fail(c, GF_ERR_ARG, "gf_pack: NULL pointer");
  const Lat L = make_lat(g);
  with_type(g, [&]<typename T, int NC>() {
    hipLaunchKernelGGL((k_pack<T, NC>), dim3(blocks_for(2ull * L.vh), 4), dim3(kBlock), 0,
                       c->stream, src, (v2<T>*)dst, L);
  });
  return launch_check(c, "gf_pack");
}

gf_status gf_unpack(gf_ctx* c, const gf_geom* g, const void* src, double* dst) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_unpack");
  if (!src || !dst) return fail(c, GF_ERR_ARG, "gf_unpack: NULL pointer");
  const Lat L = make_lat(g);
  with_type(g, [&]<typename T, int NC>() {
    hipLaunchKernelGGL((k_unpack<T, NC>), dim3(blocks_for(2ull * L.vh), 4), dim3(kBlock), 0,
                       c->stream, (const v2<T>*)src, dst, L);
  });
  return launch_check(c, "gf_unpack");
}

template <typename Ts, int NCs>
static void launch_convert_to(gf_ctx* c, const gf_geom* d, const void* src, void* dst,
                              const Lat& L, int reunit) {
  with_type(d, [&]<typename Td, int NCd>() {
    hipLaunchKernelGGL((k_convert<Ts, NCs, Td, NCd>), dim3(blocks_for(L.vh), 8), dim3(kBlock), 0,
                       c->stream, (const v2<Ts>*)src, (v2<Td>*)dst, L.vh, L.vp, reunit);
  });
}

gf_status gf_convert(gf_ctx* c, const gf_geom* s, const void* src, const gf_geom* d, void* dst,
                     int32_t reunitarize) {
  CHECK_CTX(c);
  CHECK_GEOM(c, s, "gf_convert(src)");
  CHECK_GEOM(c, d, "gf_convert(dst)");
  if (!same_extents(s, d)) return fail(c, GF_ERR_ARG, "gf_convert: extents differ");
  if (!src || !dst) return fail(c, GF_ERR_ARG, "gf_convert: NULL pointer");
  const size_t bs = gf_field_bytes(s), bd = gf_field_bytes(d);
  const char *ps = (const char*)src, *pd = (const char*)dst;
  if (ps < pd + bd && pd < ps + bs) return fail(c, GF_ERR_ARG, "gf_convert: buffers overlap");
  const Lat L = make_lat(s);
  with_type(s, [&]<typename Ts, int NCs>() {
    launch_convert_to<Ts, NCs>(c, d, src, dst, L, reunitarize ? 1 : 0);
  });
  return launch_check(c, "gf_convert");
}

size_t gf_gauge_bytes(const gf_geom* geom) {
  if (!geom_ok(geom)) return 0;
  const uint64_t V = (uint64_t)geom->nt * geom->nz * geom->ny * geom->nx;
  return (size_t)(2 * 6 * padded_half(V / 2) * 2 * sizeof(float));
}

gf_status gf_gauge_unit(gf_ctx* c, const gf_geom* g, void* G) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_gauge_unit");
  if (!G) return fail(c, GF_ERR_ARG, "gf_gauge_unit: NULL pointer");
  const Lat L = make_lat(g);
  hipLaunchKernelGGL((k_fill_unit<float, 6, 1>), dim3(blocks_for(L.vp), 2), dim3(kBlock), 0,
                     c->stream, (v2<float>*)G, L.vp);
  return launch_check(c, "gf_gauge_unit");
}

gf_status gf_gauge_pack(gf_ctx* c, const gf_geom* g, const double* src, void* G) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_gauge_pack");
  if (!src || !G) return fail(c, GF_ERR_ARG, "gf_gauge_pack: NULL pointer");
  const Lat L = make_lat(g);
  hipLaunchKernelGGL((k_pack_gauge<float>), dim3(blocks_for(2ull * L.vh)), dim3(kBlock), 0,
                     c->stream, src, (v2<float>*)G, L);
  return launch_check(c, "gf_gauge_pack");
}

gf_status gf_gauge_unpack(gf_ctx* c, const gf_geom* g, const void* G, double* dst) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_gauge_unpack");
  if (!G || !dst) return fail(c, GF_ERR_ARG, "gf_gauge_unpack: NULL pointer");
  const Lat L = make_lat(g);
  hipLaunchKernelGGL((k_unpack_gauge<float>), dim3(blocks_for(2ull * L.vh)), dim3(kBlock), 0,
                     c->stream, (const v2<float>*)G, dst, L);
  return launch_check(c, "gf_gauge_unpack");
}

gf_status gf_reunitarize(gf_ctx* c, void* U, const gf_geom* g) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_reunitarize");
  if (!U) return fail(c, GF_ERR_ARG, "gf_reunitarize: NULL pointer");
  const Lat L = make_lat(g);
  with_type(g, [&]<typename T, int NC>() {
    hipLaunchKernelGGL((k_reunitarize<T, NC>), dim3(blocks_for(L.vh), 8), dim3(kBlock), 0,
                       c->stream, (v2<T>*)U, L.vh, L.vp);
  });
  return launch_check(c, "gf_reunitarize");
}

// the measurement kernels with the per-block partial sums in `partial`
// (2 * blocks_for(st) * nt doubles)
static gf_status measure_launch(gf_ctx* c, const void* U, const gf_geom* g, int32_t gauge,
                                double* F, double* th, double* partial) {
  const Lat L = make_lat(g);
  const uint32_t bpt = blocks_for(L.st);
  const dim3 grid(bpt, L.nt);
  with_type(g, [&]<typename T, int NC>() {
    if (gauge == GF_LANDAU)
      hipLaunchKernelGGL((k_measure<T, NC, kLandau>), grid, dim3(kBlock), 0, c->stream,
                         (const v2<T>*)U, L, partial);
    else if (gauge == GF_COULOMB)
      hipLaunchKernelGGL((k_measure<T, NC, kCoulomb>), grid, dim3(kBlock), 0, c->stream,
                         (const v2<T>*)U, L, partial);
    else
      hipLaunchKernelGGL((k_measure_mag<T, NC>), grid, dim3(kBlock), 0, c->stream,
                         (const v2<T>*)U, L, partial);
  });
  const double V = 2.0 * L.vh, Vs = V / L.nt;
  if (gauge != GF_COULOMB)
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, c->stream, (const double*)partial,
                       bpt * L.nt, 12.0 * V, 3.0 * V, F, th);
  else
    hipLaunchKernelGGL(k_finish, dim3(L.nt), dim3(kBlock), 0, c->stream,
                       (const double*)partial, bpt, 9.0 * Vs, 3.0 * Vs, F, th);
  return launch_check(c, "gf_measure");
}

static size_t measure_partials(const gf_geom* g) {
  const Lat L = make_lat(g);
  return (size_t)2 * blocks_for(L.st) * L.nt;
}

gf_status measure_impl(gf_ctx* c, const void* U, const gf_geom* g, int32_t gauge, double* F,
                       double* th) {
  gf_status st = ensure_partial(c, measure_partials(g));
  if (st != GF_OK) return st;
  return measure_launch(c, U, g, gauge, F, th, c->partial);
}

gf_status gf_measure(gf_ctx* c, const void* U, const gf_geom* g, int32_t gauge, double* F,
                     double* th) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_measure");
  if (gauge != GF_LANDAU && gauge != GF_COULOMB && gauge != GF_MAG)
    return fail(c, GF_ERR_ARG, "gf_measure: bad gauge");
  if (!U || (!F && !th)) return fail(c, GF_ERR_ARG, "gf_measure: NULL pointer");
  return measure_impl(c, U, g, gauge, F, th);
}

// ---------------------------------------------------------------------------
// measurement without allocation: the partial sums go to a fixed device array
// of this library, one per GPU, for callers that cannot allocate
// ---------------------------------------------------------------------------
constexpr size_t kScratchDoubles = (size_t)1 << 19;  // 4 MiB per device
static __device__ __align__(256) double scratch[kScratchDoubles];

// device address of `scratch` on each device, looked up once per device at
// context creation with that device current (the array's name in host code is
// a host-side stand-in, not a device address)
constexpr int kScratchDevices = 64;
static double* g_scratch_ptr[kScratchDevices];
static std::mutex g_scratch_mu;

static gf_status scratch_setup(int device) {
  if (device < 0 || device >= kScratchDevices) return GF_OK;  // no static scratch there
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return GF_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(nullptr, GF_ERR_HIP, "gf_create: hipGetSymbolAddress(scratch) on device %d: %s",
                device, hipGetErrorString(e));
  g_scratch_ptr[device] = (double*)p;
  return GF_OK;
}

gf_status gf_measure_static(gf_ctx* c, const void* U, const gf_geom* g, int32_t gauge, double* F,
                            double* th) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_measure_static");
  if (gauge != GF_LANDAU && gauge != GF_COULOMB && gauge != GF_MAG)
    return fail(c, GF_ERR_ARG, "gf_measure_static: bad gauge");
  if (!U || (!F && !th)) return fail(c, GF_ERR_ARG, "gf_measure_static: NULL pointer");
  const size_t need = measure_partials(g);
  if (need > kScratchDoubles)
    return fail(c, GF_ERR_ARG,
                "gf_measure_static: the lattice needs %zu partial sums, the static scratch holds "
                "%zu (about 2^27 sites); use gf_measure",
                need, kScratchDoubles);
  double* p = (c->device >= 0 && c->device < kScratchDevices) ? g_scratch_ptr[c->device] : nullptr;
  if (!p) return fail(c, GF_ERR_UNSUPPORTED, "gf_measure_static: no static scratch on device %d",
                      c->device);
  return measure_launch(c, U, g, gauge, F, th, p);
}

gf_status gf_functional(gf_ctx* c, const void* U, const gf_geom* g, int32_t gauge, double* F) {
  if (!F) return fail(c, GF_ERR_ARG, "gf_functional: NULL output");
  return gf_measure(c, U, g, gauge, F, nullptr);
}

gf_status gf_theta(gf_ctx* c, const void* U, const gf_geom* g, int32_t gauge, double* th) {
  if (!th) return fail(c, GF_ERR_ARG, "gf_theta: NULL output");
  return gf_measure(c, U, g, gauge, nullptr, th);
}

gf_status gf_plaquette(gf_ctx* c, const void* U, const gf_geom* g, double* P) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_plaquette");
  if (!U || !P) return fail(c, GF_ERR_ARG, "gf_plaquette: NULL pointer");
  const Lat L = make_lat(g);
  const uint32_t nb = blocks_for(L.vh);
  gf_status st = ensure_partial(c, (size_t)2 * nb);
  if (st != GF_OK) return st;
  with_type(g, [&]<typename T, int NC>() {
    hipLaunchKernelGGL((k_plaquette<T, NC>), dim3(nb), dim3(kBlock), 0, c->stream,
                       (const v2<T>*)U, L, c->partial);
  });
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, c->stream, (const double*)c->partial, nb,
                     6.0 * 2.0 * L.vh, 1.0, P, (double*)nullptr);
  return launch_check(c, "gf_plaquette");
}

gf_status gf_philox(gf_ctx* c, const uint32_t* ctr, uint64_t seed, uint32_t* out, int64_t n) {
  CHECK_CTX(c);
  if (!ctr || !out || n < 0) return fail(c, GF_ERR_ARG, "gf_philox: bad arguments");
  if (n == 0) return GF_OK;
  hipLaunchKernelGGL(k_philox, dim3(blocks_for((uint64_t)n)), dim3(kBlock), 0, c->stream, ctr, out,
                     n, (uint32_t)seed, (uint32_t)(seed >> 32));
  return launch_check(c, "gf_philox");
}

// ---------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------
static int tps_ok(int32_t t) { return t == 1 || t == 2 || t == 4; }
static int ps_ok(int32_t prec, int32_t storage) {
  return (prec == GF_FP32 || prec == GF_FP64) && (storage == GF_R12 || storage == GF_R18);
}

static gf_status set_variant(gf_ctx* c, int kind, int32_t prec, int32_t storage, int32_t tps,
                             int32_t nontemporal, const char* what) {
  if (!c) return GF_ERR_ARG;
  if (!ps_ok(prec, storage)) return fail(c, GF_ERR_ARG, "%s: bad precision or storage", what);
  if (tps != 0 && !tps_ok(tps)) return fail(c, GF_ERR_ARG, "%s: tps must be 0, 1, 2 or 4", what);
  if (nontemporal < -1 || nontemporal > 2)
    return fail(c, GF_ERR_ARG, "%s: nontemporal must be -1, 0, 1 or 2", what);
  for (int cls = 0; cls < 2; ++cls) {
    ctx_var(c, kind, prec, storage, cls).tps = tps;
    ctx_var(c, kind, prec, storage, cls).nt = nontemporal;
  }
  return GF_OK;
}

gf_status gf_set_sweep_variant(gf_ctx* c, int32_t prec, int32_t storage, int32_t tps,
                               int32_t nontemporal) {
  return set_variant(c, kSweepKind, prec, storage, tps, nontemporal, "gf_set_sweep_variant");
}

gf_status gf_set_anneal_variant(gf_ctx* c, int32_t prec, int32_t storage, int32_t tps,
                                int32_t nontemporal) {
  return set_variant(c, kAnnealKind, prec, storage, tps, nontemporal, "gf_set_anneal_variant");
}

gf_status gf_sweep_variant_for(gf_ctx* c, const gf_geom* g, int32_t* tps, int32_t* nontemporal) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_sweep_variant_for");
  if (!tps || !nontemporal) return fail(c, GF_ERR_ARG, "gf_sweep_variant_for: NULL pointer");
  *tps = ctx_tps(c, g);
  *nontemporal = ctx_nt(c, g);
  return GF_OK;
}

gf_status gf_anneal_variant_for(gf_ctx* c, const gf_geom* g, int32_t* tps, int32_t* nontemporal) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_anneal_variant_for");
  if (!tps || !nontemporal) return fail(c, GF_ERR_ARG, "gf_anneal_variant_for: NULL pointer");
  *tps = ctx_tps(c, g, kAnnealKind);
  *nontemporal = ctx_nt(c, g, kAnnealKind);
  return GF_OK;
}

gf_status gf_get_sweep_variant(gf_ctx* c, int32_t prec, int32_t storage, int32_t* tps,
                               int32_t* nontemporal) {
  if (!c || !tps || !nontemporal) return GF_ERR_ARG;
  if (!ps_ok(prec, storage)) return fail(c, GF_ERR_ARG, "gf_get_sweep_variant: bad precision or storage");
  gf_geom g = {2, 2, 2, 2, prec, storage};
  *tps = ctx_tps(c, &g);
  *nontemporal = ctx_nt(c, &g);
  return GF_OK;
}

namespace {

// The autotuner's timing, done the way the drivers run the kernels: for each
// of the nine variants (lanes per site 1, 2, 4 x nontemporal mode 0, 1, 2) a
// block of `reps` units of work (`unit` enqueues one: a RED/BLACK sweep pair,
// or an annealing step) followed by `tail` (the drivers' check between
// blocks) is captured as a hipGraph on the scratch field; the
// nine graphs are then replayed in turn, round after round, and each variant
// is timed by the median of its rounds, so that slow drifts and the order of
// the variants weigh on all of them alike. Returns the median ms per unit in
// times[9] (index 3 * mode + log2(lanes)).
template <class Unit, class Tail>
gf_status tune_variants(gf_ctx* c, int kind, const gf_geom* g, Unit&& unit, Tail&& tail,
                        int half_sweeps_per_unit, float times[kVariants]) {
  const int i64 = g->prec == GF_FP64, i18 = g->storage == GF_R18;
  const int cls = size_class(gf_field_bytes(g));
  gf_ctx::Variant saved = c->var[kind][i64][i18][cls];
  gf_status st = GF_OK;
  // size of a block: 100 units, the drivers' check interval, capped at about
  // 100 ms of work (one timed unit of the built-in variant sets the cap); with
  // blocks of a few ms the stores-streamed variants timed up to 2% faster
  // than they then ran between the checks of a fix at 32^4
  float ms1 = 0;
  if ((st = unit()) != GF_OK) return st;
  HIP_OR_FAIL(c, hipEventRecord(c->ev[0], c->stream));
  if ((st = unit()) != GF_OK) return st;
  HIP_OR_FAIL(c, hipEventRecord(c->ev[1], c->stream));
  HIP_OR_FAIL(c, hipEventSynchronize(c->ev[1]));
  HIP_OR_FAIL(c, hipEventElapsedTime(&ms1, c->ev[0], c->ev[1]));
  const int reps = std::max(2, std::min(100, (int)std::ceil(100.0 / std::max(ms1, 1e-3f))));
  TuneGraph graphs[kVariants];
  for (int k = 0; k < kVariants && st == GF_OK; ++k) {
    c->var[kind][i64][i18][cls].tps = 1 << (k % 3);
    c->var[kind][i64][i18][cls].nt = k / 3;
    st = capture_block(c, [&]() -> gf_status {
      for (int r = 0; r < reps; ++r) {
        gf_status s2 = unit();
        if (s2 != GF_OK) return s2;
      }
      return tail();
    }, graphs[k]);
  }
  c->var[kind][i64][i18][cls] = saved;
  if (st != GF_OK) return st;
  constexpr int kRounds = 5;
  float t[kVariants][kRounds];
  for (int k = 0; k < kVariants; ++k) HIP_OR_FAIL(c, hipGraphLaunch(graphs[k].exec, c->stream));  // warm-up
  for (int r = 0; r < kRounds; ++r)
    for (int k = 0; k < kVariants; ++k)
      if ((st = time_replay(c, graphs[k], &t[k][r])) != GF_OK) return st;
  for (int k = 0; k < kVariants; ++k) {
    std::sort(t[k], t[k] + kRounds);
    times[k] = t[k][kRounds / 2] / (float)(reps * half_sweeps_per_unit);
  }
  return GF_OK;
}

// scratch copy of U_like (or the unit field) for the tuner
gf_status tune_scratch(gf_ctx* c, const gf_geom* g, const void* U_like, void** out) {
  const size_t bytes = gf_field_bytes(g);
  HIP_OR_FAIL(c, hipMalloc(out, bytes));
  const Lat L = make_lat(g);
  if (U_like) {
    if (hipMemcpyAsync(*out, U_like, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
      (void)hipFree(*out);
      *out = nullptr;
      return fail(c, GF_ERR_HIP, "autotune: copy of the sample field failed");
    }
  } else {
    with_type(g, [&]<typename T, int NC>() {
      hipLaunchKernelGGL((k_fill_unit<T, NC, 4>), dim3(blocks_for(L.vp), 8), dim3(kBlock), 0,
                         c->stream, (v2<T>*)*out, L.vp);
    });
  }
  return GF_OK;
}

// keep the fastest variant for g's precision, storage and size class
void keep_fastest(gf_ctx* c, int kind, const gf_geom* g, const float times[kVariants],
                  int32_t* tps_out, int32_t* nt_out, float* ms_out) {
  int best = 0;
  for (int k = 1; k < kVariants; ++k)
    if (times[k] < times[best]) best = k;
  const int cls = size_class(gf_field_bytes(g));
  ctx_var(c, kind, g->prec, g->storage, cls).tps = 1 << (best % 3);
  ctx_var(c, kind, g->prec, g->storage, cls).nt = best / 3;
  if (tps_out) *tps_out = 1 << (best % 3);
  if (nt_out) *nt_out = best / 3;
  if (ms_out)
    for (int k = 0; k < kVariants; ++k) ms_out[k] = times[k];
}

}  // namespace

gf_status gf_autotune(gf_ctx* c, const gf_geom* g, int32_t gauge, const void* U_like,
                      int32_t* tps_out, int32_t* nt_out, float* ms_out) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_autotune");
  if (gauge != GF_LANDAU && gauge != GF_COULOMB && gauge != GF_MAG)
    return fail(c, GF_ERR_ARG, "gf_autotune: bad gauge");
  void* scratch = nullptr;
  gf_status st = tune_scratch(c, g, U_like, &scratch);
  if (st != GF_OK) return st;
  float times[kVariants] = {};
  // the drivers' check after each block: reunitarisation, F and theta (the
  // partial sums and outputs allocated before the capture)
  const int nout = gauge == GF_COULOMB ? g->nt : 1;
  if ((st = ensure_partial(c, measure_partials(g))) == GF_OK) st = ensure_out(c, nout);
  if (st == GF_OK)
    st = tune_variants(
        c, kSweepKind, g,
        [&]() -> gf_status {
          gf_status s2 = gf_sweep(c, scratch, g, gauge, 0, 1.7);
          return s2 != GF_OK ? s2 : gf_sweep(c, scratch, g, gauge, 1, 1.7);
        },
        [&]() -> gf_status {
          gf_status s2 = gf_reunitarize(c, scratch, g);
          return s2 != GF_OK ? s2
                             : measure_launch(c, scratch, g, gauge, c->dev_out, c->dev_out + c->out_cap,
                                              c->partial);
        },
        2, times);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(scratch);
  if (st != GF_OK) return st;
  keep_fastest(c, kSweepKind, g, times, tps_out, nt_out, ms_out);
  return GF_OK;
}

gf_status gf_autotune_anneal(gf_ctx* c, const gf_geom* g, int32_t gauge, const void* U_like,
                             double T, int32_t* tps_out, int32_t* nt_out, float* ms_out) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_autotune_anneal");
  if (gauge != GF_LANDAU && gauge != GF_COULOMB)
    return fail(c, GF_ERR_ARG, "gf_autotune_anneal: gauge must be GF_LANDAU or GF_COULOMB");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(c, GF_ERR_ARG, "gf_autotune_anneal: T must be > 0");
  void* scratch = nullptr;
  gf_status st = tune_scratch(c, g, U_like, &scratch);
  if (st != GF_OK) return st;
  float times[kVariants] = {};
  // one step: heatbath RED and BLACK at T, one microcanonical sweep; the
  // step index is fixed, so every replay draws the same numbers
  st = tune_variants(
      c, kAnnealKind, g,
      [&]() -> gf_status {
        gf_status s2 = GF_OK;
        for (int p = 0; p < 2 && s2 == GF_OK; ++p) s2 = gf_heatbath_half(c, scratch, g, gauge, p, T, 1, 0);
        for (int p = 0; p < 2 && s2 == GF_OK; ++p) s2 = gf_micro_half(c, scratch, g, gauge, p);
        return s2;
      },
      []() -> gf_status { return GF_OK; }, 4, times);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(scratch);
  if (st != GF_OK) return st;
  keep_fastest(c, kAnnealKind, g, times, tps_out, nt_out, ms_out);
  return GF_OK;
}

gf_status gf_autotune_storage(gf_ctx* c, const gf_geom* g, int32_t gauge, const double* U_canon,
                              int32_t* storage_out, float* ms_out) {
  CHECK_CTX(c);
  CHECK_GEOM(c, g, "gf_autotune_storage");
  if (!U_canon || !storage_out) return fail(c, GF_ERR_ARG, "gf_autotune_storage: NULL pointer");
  float best[2] = {0, 0};
  const int32_t storages[2] = {GF_R12, GF_R18};
  for (int k = 0; k < 2; ++k) {
    gf_geom gs = *g;
    gs.storage = storages[k];
    void* f = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&f, gf_field_bytes(&gs)));
    gf_status st = gf_pack(c, &gs, U_canon, f);
    float ms[kVariants] = {};
    if (st == GF_OK) st = gf_autotune(c, &gs, gauge, f, nullptr, nullptr, ms);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(f);
    if (st != GF_OK) return st;
    best[k] = *std::min_element(ms, ms + kVariants);
  }
  *storage_out = best[1] < best[0] ? GF_R18 : GF_R12;
  if (ms_out) {
    ms_out[0] = best[0];
    ms_out[1] = best[1];
  }
  return GF_OK;
}

gf_status gf_stream_probe(gf_ctx* c, const void* src, void* dst, size_t bytes, int32_t kind) {
  CHECK_CTX(c);
  if (!dst || (kind != 1 && !src) || (bytes % 16) != 0 || kind < 0 || kind > 2)
    return fail(c, GF_ERR_ARG, "gf_stream_probe: bad arguments");
  const size_t n = bytes / 16;
  if (n == 0) return GF_OK;
  if (n > ((size_t)1 << 36)) return fail(c, GF_ERR_ARG, "gf_stream_probe: too large");
  const unsigned grid = blocks_for(n);
  if (kind == 2 && bytes < (size_t)grid * sizeof(double))
    return fail(c, GF_ERR_ARG, "gf_stream_probe: dst too small for the partial sums");
  if (kind == 0)
    hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(kBlock), 0, c->stream, (const double2*)src,
                       (double2*)dst, n);
  else if (kind == 1)
    hipLaunchKernelGGL(k_probe_rmw, dim3(grid), dim3(kBlock), 0, c->stream, (v2<double>*)dst, n);
  else
    hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(kBlock), 0, c->stream, (const double2*)src,
                       (double*)dst, n);
  return launch_check(c, "gf_stream_probe");
}
