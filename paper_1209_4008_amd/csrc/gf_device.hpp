// gf_device.hpp -- device building blocks of libgf (gfx950).
//
// Complex arithmetic with explicit fused multiply-adds, SU(3) links held in
// registers, the parity-split site-fastest device layout, index arithmetic of
// the periodic 4D lattice, and the Philox4x32-10 generator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gf {

// ---------------------------------------------------------------------------
// scalar traits
// ---------------------------------------------------------------------------
template <typename T>
struct V2T;
template <>
struct V2T<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct V2T<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <typename T>
using v2 = typename V2T<T>::type;

// 1/sqrt(x) for positive normal x. FP32: the hardware estimate (1 ulp).
// FP64: the hardware estimate refined by two Newton steps for y = x^(-1/2),
// y <- y (3/2 - x y^2 / 2), each of which squares the relative error.
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  double e = fma(-hx * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-hx * y, y, 0.5);
  return fma(y, e, y);
}
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }

// |w|^2 below which a subgroup is skipped (the transformation is undefined).
template <typename T>
struct Tiny;
template <>
struct Tiny<float> {
  static constexpr float value = 1e-30f;
};
template <>
struct Tiny<double> {
  static constexpr double value = 4e-300;
};

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <typename T>
struct Cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ Cx<T> cx(T re, T im) {
  Cx<T> z;
  z.re = re;
  z.im = im;
  return z;
}
template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) {
  return cx(a.re + b.re, a.im + b.im);
}
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) {
  return cx(a.re - b.re, a.im - b.im);
}
template <typename T>
__device__ __forceinline__ Cx<T> cconj(Cx<T> a) {
  return cx(a.re, -a.im);
}
// a*b
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return cx(fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re));
}
// c + a*b
template <typename T>
__device__ __forceinline__ Cx<T> cmac(Cx<T> c, Cx<T> a, Cx<T> b) {
  return cx(fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im)));
}
// c + a*conj(b)
template <typename T>
__device__ __forceinline__ Cx<T> cmac_cb(Cx<T> c, Cx<T> a, Cx<T> b) {
  return cx(fma(a.re, b.re, fma(a.im, b.im, c.re)), fma(a.im, b.re, fma(-a.re, b.im, c.im)));
}
// conj(a*b - c*d)
template <typename T>
__device__ __forceinline__ Cx<T> cross_term(Cx<T> a, Cx<T> b, Cx<T> c, Cx<T> d) {
  Cx<T> r = cmul(a, b);
  r = cx(r.re - (c.re * d.re - c.im * d.im), r.im - (c.re * d.im + c.im * d.re));
  return cconj(r);
}

// ---------------------------------------------------------------------------
// SU(3) link in registers
// ---------------------------------------------------------------------------
template <typename T>
struct Su3 {
  Cx<T> e[3][3];
};

template <typename T>
__device__ __forceinline__ void set_zero(Su3<T>& A) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) A.e[a][b] = cx<T>(0, 0);
}
template <typename T>
__device__ __forceinline__ void set_unit(Su3<T>& A) {
  set_zero(A);
#pragma unroll
  for (int a = 0; a < 3; ++a) A.e[a][a] = cx<T>(1, 0);
}

// row 2 of an SU(3) matrix from rows 0 and 1: conj(row0 x row1)
template <typename T>
__device__ __forceinline__ void rebuild_row2(Su3<T>& A) {
  A.e[2][0] = cross_term(A.e[0][1], A.e[1][2], A.e[0][2], A.e[1][1]);
  A.e[2][1] = cross_term(A.e[0][2], A.e[1][0], A.e[0][0], A.e[1][2]);
  A.e[2][2] = cross_term(A.e[0][0], A.e[1][1], A.e[0][1], A.e[1][0]);
}

// ---------------------------------------------------------------------------
// device layout. The sites of one parity p (half index h) are cut into tiles
// of kTile; a tile holds the links of its sites direction after direction,
// and each link's NC components one after another, kTile elements each:
//   elem(p, mu, c, h) = p*4*NC*vp + (h/kTile)*kTile*4*NC + (mu*NC + c)*kTile
//                       + h%kTile
// vp = V/2 rounded up to a multiple of kTile; the padding sites of the last
// tile belong to no lattice site and are never read by a site update. A wave
// reading one component of 16..64 consecutive sites reads one contiguous run,
// and the forward links of a tile (4*NC runs) lie in one contiguous region,
// so the many concurrent streams of a half-sweep touch few DRAM pages.
// 2048 sites per tile hold a whole z plane of lattices up to 64^2 x-y sites
// (1152 half-sites at 48^4), so the y and z backward neighbours of a block's
// sites mostly lie in the block's own tile; measured against tiles of 64 to
// 16384 sites it sweeps lattices of 32^4 to 56^4 fastest (48^4 FP64 12 reals
// 8% faster than 128-site tiles, 56^4 12%), while lattices of 24^4 and below
// lose 2-5% of a 10-40 us half-sweep.
// Fields with one matrix per site (the gauge transformation, ND = 1) use the
// same scheme with the direction dropped.
// ---------------------------------------------------------------------------
constexpr uint32_t kTile = 2048;

__host__ __device__ constexpr uint64_t padded_half(uint64_t vh) {
  return (vh + kTile - 1) / kTile * kTile;
}

// offset of component 0 of link (p, mu) at half index h; the components
// follow at strides of kTile
template <int NC, int ND = 4>
__host__ __device__ __forceinline__ size_t link_offset(uint32_t vp, int p, int mu, uint32_t h) {
  return (size_t)p * ND * NC * vp + (size_t)(h & ~(kTile - 1)) * ND * NC +
         (size_t)(mu * NC) * kTile + (h & (kTile - 1));
}

// Nontemporal modes of the link accesses, a tuning axis of the sweep kernels.
// Each link is read and written once per half-sweep, so there is no reuse
// inside a launch; what pays depends on how much of the field the Infinity
// Cache keeps between half-sweeps:
//   kNTNone    ordinary loads and stores,
//   kNTAll     loads and stores streamed (fields far larger than the cache),
//   kNTStores  stores streamed, loads cached (fields the cache partly holds).
constexpr int kNTNone = 0, kNTAll = 1, kNTStores = 2;

#ifdef GF_ACCESS_COUNT
// Access-count builds only (the debug library that checks the RED/BLACK
// decomposition): every element a link load or store touches is counted in a
// shadow array, at the element's offset from the start of its field; two
// fields (the links and the gauge-transformation field).
struct AccessCount {
  const char* base[2];
  size_t bytes[2];
  unsigned* reads[2];
  unsigned* writes[2];
};
static __device__ AccessCount gf_access_count;

template <typename T>
__device__ __forceinline__ void count_access(const v2<T>* p, bool write) {
  const char* c = (const char*)p;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const char* b = gf_access_count.base[r];
    if (b && c >= b && c < b + gf_access_count.bytes[r]) {
      unsigned* cnt = write ? gf_access_count.writes[r] : gf_access_count.reads[r];
      atomicAdd(cnt + (size_t)(c - b) / sizeof(v2<T>), 1u);
    }
  }
}
#define GF_COUNT_ACCESS(T, p, w) count_access<T>((p), (w))
#else
#define GF_COUNT_ACCESS(T, p, w) ((void)0)
#endif

// q points at component 0 of the link.
template <typename T, int NC, int NT = kNTNone>
__device__ __forceinline__ void load_link(const v2<T>* __restrict__ q, Su3<T>& A) {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const v2<T>* p = q + c * kTile;
    GF_COUNT_ACCESS(T, p, false);
    const v2<T> v = (NT == kNTAll) ? __builtin_nontemporal_load(p) : *p;
    A.e[c / 3][c % 3] = cx<T>(v.x, v.y);
  }
  if (NC == 6) rebuild_row2(A);
}

template <typename T, int NC, int NT = kNTNone>
__device__ __forceinline__ void store_link(v2<T>* __restrict__ q, const Su3<T>& A) {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    v2<T> v;
    v.x = A.e[c / 3][c % 3].re;
    v.y = A.e[c / 3][c % 3].im;
    v2<T>* p = q + c * kTile;
    GF_COUNT_ACCESS(T, p, true);
    if (NT != kNTNone)
      __builtin_nontemporal_store(v, p);
    else
      *p = v;
  }
}

// ---------------------------------------------------------------------------
// exact unsigned division by a runtime constant (Granlund & Montgomery 1994,
// Thm 4.2: m = ceil(2^(32+l)/d), l = ceil(log2 d); floor(n*m / 2^(32+l)) =
// floor(n/d) for all n < 2^32). m < 2^33 and n < 2^31 keep n*m < 2^64.
// ---------------------------------------------------------------------------
struct FastDiv {
  uint64_t m;
  uint32_t shift;
  uint32_t d;
};

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((uint64_t)n * f.m) >> f.shift);
}

// ---------------------------------------------------------------------------
// lattice geometry in half indices
// ---------------------------------------------------------------------------
struct Lat {
  uint32_t nt, nz, ny, nx;
  uint32_t hx;           // nx / 2
  uint32_t vh;           // V / 2
  uint32_t vp;           // V / 2 rounded up to a multiple of kTile (block stride unit)
  uint32_t sy, sz, st;   // half-index strides of y, z, t: hx, ny*hx, nz*ny*hx
  FastDiv div_hx, div_ny, div_nz;
};

struct Site {
  uint32_t t, z, y, x;
  uint32_t xodd;  // x & 1
};

// coordinates of the site of parity p with half index h
__host__ __device__ __forceinline__ Site site_of(const Lat& L, uint32_t h, int p) {
  Site S;
  const uint32_t r = fdiv(h, L.div_hx);  // (t*nz + z)*ny + y
  const uint32_t xh = h - r * L.hx;
  const uint32_t r2 = fdiv(r, L.div_ny);
  S.y = r - r2 * L.ny;
  S.t = fdiv(r2, L.div_nz);
  S.z = r2 - S.t * L.nz;
  S.xodd = (uint32_t)(p + S.t + S.z + S.y) & 1u;
  S.x = 2 * xh + S.xodd;
  return S;
}

// half index of x - mu (a site of the other parity)
__host__ __device__ __forceinline__ uint32_t back_h(const Lat& L, uint32_t h, const Site& S, int mu) {
  switch (mu) {
    case 0:
      return S.t ? h - L.st : h + (L.nt - 1) * L.st;
    case 1:
      if (S.xodd) return h;
      return (S.x != 0) ? h - 1 : h + L.hx - 1;
    case 2:
      return S.y ? h - L.sy : h + (L.ny - 1) * L.sy;
    default:
      return S.z ? h - L.sz : h + (L.nz - 1) * L.sz;
  }
}

// half index of x + mu (a site of the other parity)
__host__ __device__ __forceinline__ uint32_t fwd_h(const Lat& L, uint32_t h, const Site& S, int mu) {
  switch (mu) {
    case 0:
      return (S.t + 1 < L.nt) ? h + L.st : h - (L.nt - 1) * L.st;
    case 1:
      if (!S.xodd) return h;
      return (S.x + 1 < L.nx) ? h + 1 : h - (L.hx - 1);
    case 2:
      return (S.y + 1 < L.ny) ? h + L.sy : h - (L.ny - 1) * L.sy;
    default:
      return (S.z + 1 < L.nz) ? h + L.sz : h - (L.nz - 1) * L.sz;
  }
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t v[4];
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// uniform in (0, 1): (u + 1/2) 2^-32, formed in T
template <typename T>
__device__ __forceinline__ T unit_open(uint32_t u) {
  return ((T)u + (T)0.5) * (T)2.3283064365386962890625e-10;
}

}  // namespace gf
