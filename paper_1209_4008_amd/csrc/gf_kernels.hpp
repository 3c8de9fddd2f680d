// gf_kernels.hpp -- HIP kernels of libgf for gfx950 (wave64, no MFMA: 3x3
// complex products are far too small to be a dense contraction; the sweep is
// bound by HBM traffic).
//
// Site update (Alg. 1 of the paper) as computed here:
//   gather the 8 links of x (4 forward from the block of x's parity, 4
//   backward from the other parity's block), K = sum_{mu in D} U_mu(x) +
//   U_mu(x-mu)^dag (eq. (5) with the neighbours' transformations already in
//   the links); for the subgroups (0,1), (0,2), (1,2): w = 2 x quaternion part
//   of the (i,j) block of K^dag (whose normalisation is the local maximum of
//   eq. (6)), s = update(w), K <- G(s) K and Gtot <- G(s) Gtot; finally
//   U_mu(x) <- Gtot U_mu(x), U_mu(x-mu) <- U_mu(x-mu) Gtot^dag for all mu.
// K <- G K is exact algebra (the links after the subgroup step sum to G K),
// so this equals applying each subgroup to the 8 links in turn, with 1/3 of
// the link arithmetic. Every link is read once and written once per
// half-sweep.
#pragma once

#include "gf_device.hpp"

namespace gf {

constexpr int kBlock = 256;
constexpr int kLandau = 0;
constexpr int kCoulomb = 1;
constexpr int kMAG = 2;  // maximally Abelian gauge (its own site update, k_mag_half)

template <int GAUGE>
struct FirstDir {
  static constexpr int value = (GAUGE == kCoulomb) ? 1 : 0;
};

// ---------------------------------------------------------------------------
// subgroup algebra
// ---------------------------------------------------------------------------
// w = 2 x quaternion part of the (I,J) block of K^dagger, for the convention
// a <-> [[a0 + i a3, a2 + i a1], [-a2 + i a1, a0 - i a3]]
template <typename T, int I, int J>
__device__ __forceinline__ void subgroup_w(const Su3<T>& K, T w[4]) {
  w[0] = K.e[I][I].re + K.e[J][J].re;
  w[1] = -(K.e[I][J].im + K.e[J][I].im);
  w[2] = K.e[J][I].re - K.e[I][J].re;
  w[3] = K.e[J][J].im - K.e[I][I].im;
}

// M <- G(s) M on rows I, J
template <typename T, int I, int J>
__device__ __forceinline__ void left_su2(Su3<T>& M, const T s[4]) {
  const Cx<T> gii = cx(s[0], s[3]), gij = cx(s[2], s[1]);
  const Cx<T> gji = cx(-s[2], s[1]), gjj = cx(s[0], -s[3]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const Cx<T> mi = M.e[I][k], mj = M.e[J][k];
    M.e[I][k] = cmac(cmul(gii, mi), gij, mj);
    M.e[J][k] = cmac(cmul(gji, mi), gjj, mj);
  }
}

// quaternion product for Q(a) Q(b) = Q(c)
template <typename T>
__device__ __forceinline__ void qmul(const T a[4], const T b[4], T c[4]) {
  c[0] = a[0] * b[0] - (a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
  c[1] = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);
  c[2] = a[0] * b[2] + b[0] * a[2] - (a[3] * b[1] - a[1] * b[3]);
  c[3] = a[0] * b[3] + b[0] * a[3] - (a[1] * b[2] - a[2] * b[1]);
}

// ---- update policies: w -> SU(2) quaternion s (false: leave the subgroup) ----

// Overrelaxation (Sec. 2; the form of the power whose operation count equals
// the paper's count for this step in Alg. 1):
// b = (omega w0^2 + |wv|^2)/|w|^2, c = (w0^2 + b^2 |wv|^2)^(-1/2),
// s = (c w0, b c wv); omega = 1 gives s = w/|w|.
template <typename T>
struct UpdOR {
  T omega;
  __device__ __forceinline__ bool operator()(const T w[4], uint32_t, int, T s[4]) const {
    const T a0sq = w[0] * w[0];
    const T avsq = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    const T n = a0sq + avsq;
    if (!(n > Tiny<T>::value)) return false;
    const T rn = rsqrt_t(n);
    const T b = (omega * a0sq + avsq) * (rn * rn);
    const T c = rsqrt_t(a0sq + b * b * avsq);
    const T bc = b * c;
    s[0] = c * w[0];
    s[1] = bc * w[1];
    s[2] = bc * w[2];
    s[3] = bc * w[3];
    return true;
  }
};

__device__ __forceinline__ float atan2_t(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double atan2_t(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ void sincos_t(float a, float* sn, float* cs) { sincosf(a, sn, cs); }
__device__ __forceinline__ void sincos_t(double a, double* sn, double* cs) { sincos(a, sn, cs); }

// Other forms of g^omega (Sec. 2: the power is taken to first or second
// order). With g = w/|w| = 1 + a: form 1 is 1 + omega a, form 2 is
// 1 + omega a + omega (omega - 1)/2 a^2 (a^2 = (a0^2 - |gv|^2, 2 a0 gv)), form 3
// the exact power (cos(omega phi), n sin(omega phi)) of g = (cos phi, n sin phi),
// left at g when gv = 0; the result is divided by its length.
template <typename T>
struct UpdORForm {
  T omega;
  int form;  // 1, 2 or 3 (uniform over the launch)
  __device__ __forceinline__ bool operator()(const T w[4], uint32_t, int, T s[4]) const {
    const T n2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    if (!(n2 > Tiny<T>::value)) return false;
    const T r = rsqrt_t(n2);
    const T g0 = w[0] * r, g1 = w[1] * r, g2 = w[2] * r, g3 = w[3] * r;
    const T gv2 = g1 * g1 + g2 * g2 + g3 * g3;
    T t0, f;
    if (form == 3) {
      const T nv = sqrt(gv2);
      if (!(nv > T(0))) {
        s[0] = g0;
        s[1] = g1;
        s[2] = g2;
        s[3] = g3;
        return true;
      }
      T sn, cs;
      sincos_t(omega * atan2_t(nv, g0), &sn, &cs);
      t0 = cs;
      f = sn / nv;
    } else {
      const T a0 = g0 - T(1);
      const T c2 = form == 2 ? T(0.5) * omega * (omega - T(1)) : T(0);
      t0 = T(1) + omega * a0 + c2 * (a0 * a0 - gv2);
      f = omega + T(2) * c2 * a0;
    }
    const T m2 = t0 * t0 + f * f * gv2;
    if (!(m2 > Tiny<T>::value)) return false;
    const T m = rsqrt_t(m2);
    s[0] = t0 * m;
    s[1] = f * m * g1;
    s[2] = f * m * g2;
    s[3] = f * m * g3;
    return true;
  }
};

// Microcanonical reflection: s = (w/|w|)^2, leaves Re tr[g K] unchanged.
template <typename T>
struct UpdMicro {
  __device__ __forceinline__ bool operator()(const T w[4], uint32_t, int, T s[4]) const {
    const T n2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    if (!(n2 > Tiny<T>::value)) return false;
    const T r = rsqrt_t(n2);
    const T a0 = w[0] * r;
    s[0] = a0 * a0 - (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) * (r * r);
    s[1] = 2 * a0 * (w[1] * r);
    s[2] = 2 * a0 * (w[2] * r);
    s[3] = 2 * a0 * (w[3] * r);
    return true;
  }
};

// ---------------------------------------------------------------------------
// lane exchange inside a quad (DPP quad_perm). The TPS lanes of a site are
// consecutive and aligned, so a site's lanes always sit in one quad.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ int quad_perm_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
// value of lane (l ^ MASK): quad_perm selectors xor 1 -> [1,0,3,2] = 0xB1,
// xor 2 -> [2,3,0,1] = 0x4E
template <int MASK>
__device__ __forceinline__ int quad_xor_i(int v) {
  return quad_perm_i<(MASK == 1) ? 0xB1 : 0x4E>(v);
}
template <int MASK>
__device__ __forceinline__ float quad_xor(float v) {
  return __builtin_bit_cast(float, quad_xor_i<MASK>(__builtin_bit_cast(int, v)));
}
template <int MASK>
__device__ __forceinline__ double quad_xor(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = quad_xor_i<MASK>((int)(uint32_t)b);
  const int hi = quad_xor_i<MASK>((int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// value of lane SRC of the calling lane's own site (TPS lanes per site)
template <int TPS, int SRC>
__device__ __forceinline__ int site_bcast_i(int v) {
  if constexpr (TPS == 1)
    return v;
  else if constexpr (TPS == 2)
    return quad_perm_i<SRC | (SRC << 2) | ((2 + SRC) << 4) | ((2 + SRC) << 6)>(v);
  else
    return quad_perm_i<SRC * 0x55>(v);
}
template <int TPS, int SRC>
__device__ __forceinline__ float site_bcast(float v) {
  return __builtin_bit_cast(float, site_bcast_i<TPS, SRC>(__builtin_bit_cast(int, v)));
}

// Heatbath with weight exp(Re tr[g K]/T): with g = X what, Re tr = |w| X0, so
// X0 is drawn with density ~ sqrt(1 - X0^2) exp(alpha X0), alpha = |w|/T, by
// Kennedy & Pendleton (Phys. Lett. B 156 (1985) 393), and (X1, X2, X3) is
// uniform on the sphere of radius sqrt(1 - X0^2).
// Philox: key (seed lo, seed hi), counter (site, sweep, tag, attempt),
// tag = 0x1000 | kind << 8 | subgroup, kind 0 = trial, 1 = direction.
// transcendental functions of the sampler: in FP32 the hardware
// approximations (relative error ~1e-6, below what the FP32 links and the
// FP32 accept test resolve anyway); in FP64 the correctly rounded library
// functions, which the parity tests against the oracle rely on
__device__ __forceinline__ float hb_log(float x) { return __logf(x); }
__device__ __forceinline__ double hb_log(double x) { return log(x); }
__device__ __forceinline__ float hb_cos(float x) { return __cosf(x); }
__device__ __forceinline__ double hb_cos(double x) { return cos(x); }
__device__ __forceinline__ float hb_sin(float x) { return __sinf(x); }
__device__ __forceinline__ double hb_sin(double x) { return sin(x); }

constexpr uint32_t kTagKP = 0x1000u;
constexpr uint32_t kTagDir = 0x1100u;
constexpr uint32_t kMaxAttempts = 1024u;

// The first trial and the direction of each subgroup's draw do not depend on
// the links: a site's heatbath step can draw them before its links arrive, so
// that the Philox rounds and transcendentals overlap the loads. num = the
// trial's -(log u0 + cos^2(2 pi u1) log u2), to be divided by 2 alpha.
template <typename T>
struct HBDraws {
  T num[3], u3[3], cth[3], sth[3], cph[3], sph[3];
};

template <typename T>
struct UpdHB {
  T temp;
  uint32_t k0, k1, sweep;
  // subgroup sg's first trial and direction: out = (num, u3, cos theta,
  // sin theta, cos phi, sin phi)
  __device__ __forceinline__ void draw_one(uint32_t site, uint32_t sg, T out[6]) const {
    const T two_pi = (T)6.283185307179586476925286766559;
    const U4 r = philox4x32_10(site, sweep, kTagKP | sg, 0u, k0, k1);
    const T u0 = unit_open<T>(r.v[0]), u1 = unit_open<T>(r.v[1]);
    const T u2 = unit_open<T>(r.v[2]);
    const T cs = hb_cos(two_pi * u1);
    out[0] = -(hb_log(u0) + cs * cs * hb_log(u2));
    out[1] = unit_open<T>(r.v[3]);
    const U4 q = philox4x32_10(site, sweep, kTagDir | sg, 0u, k0, k1);
    const T d0 = unit_open<T>(q.v[0]), d1 = unit_open<T>(q.v[1]);
    out[2] = 2 * d0 - 1;
    out[3] = sqrt_t(fmax(T(0), 1 - out[2] * out[2]));
    const T phi = two_pi * d1;
    out[4] = hb_cos(phi);
    out[5] = hb_sin(phi);
  }
  // the step with the first trial and the direction taken from d (the same
  // numbers operator() draws, combined in the same order). The further
  // trials are shared by the site's TPS lanes: in each round lane r tries
  // attempt att + r, and the site takes the first accepted attempt in order
  // (every lane gets the owning lane's value bit for bit).
  template <int TPS>
  __device__ __forceinline__ bool with_draws(const T w[4], uint32_t site, int sg, T s[4],
                                             const HBDraws<T>& d, int r) const {
    const T n2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    if (!(n2 > Tiny<T>::value)) return false;
    const T n = sqrt_t(n2);
    const T alpha = n / temp;
    const T two_pi = (T)6.283185307179586476925286766559;
    T lam2 = -1;
    {
      const T l2 = d.num[sg] / (2 * alpha);
      if (d.u3[sg] * d.u3[sg] <= 1 - l2) lam2 = l2;
    }
    for (uint32_t att = 1; lam2 < 0 && att < kMaxAttempts; att += TPS) {
      const uint32_t a = att + (uint32_t)r;
      T l2 = 0;
      int acc = 0;
      if (a < kMaxAttempts) {
        const U4 q = philox4x32_10(site, sweep, kTagKP | (uint32_t)sg, a, k0, k1);
        const T u0 = unit_open<T>(q.v[0]), u1 = unit_open<T>(q.v[1]);
        const T u2 = unit_open<T>(q.v[2]), u3 = unit_open<T>(q.v[3]);
        const T cs = hb_cos(two_pi * u1);
        l2 = -(hb_log(u0) + cs * cs * hb_log(u2)) / (2 * alpha);
        acc = u3 * u3 <= 1 - l2;
      }
      if constexpr (TPS == 1) {
        if (acc) lam2 = l2;
      } else {
#pragma unroll
        for (int j = TPS - 1; j >= 0; --j) {  // the earliest accepted attempt wins
          int acc_j;
          T l2_j;
          if (j == 0) {
            acc_j = site_bcast_i<TPS, 0>(acc);
            l2_j = site_bcast<TPS, 0>(l2);
          } else if (j == 1) {
            acc_j = site_bcast_i<TPS, 1>(acc);
            l2_j = site_bcast<TPS, 1>(l2);
          } else if (j == 2) {
            acc_j = site_bcast_i<TPS, (TPS > 2 ? 2 : 0)>(acc);
            l2_j = site_bcast<TPS, (TPS > 2 ? 2 : 0)>(l2);
          } else {
            acc_j = site_bcast_i<TPS, (TPS > 3 ? 3 : 0)>(acc);
            l2_j = site_bcast<TPS, (TPS > 3 ? 3 : 0)>(l2);
          }
          if (acc_j) lam2 = l2_j;
        }
      }
    }
    if (lam2 < 0) return false;  // attempt cap: subgroup left unchanged
    const T rad = 2 * sqrt_t(lam2 * (1 - lam2));
    const T X[4] = {1 - 2 * lam2, rad * d.sth[sg] * d.cph[sg], rad * d.sth[sg] * d.sph[sg],
                    rad * d.cth[sg]};
    const T wh[4] = {w[0] / n, w[1] / n, w[2] / n, w[3] / n};
    qmul(X, wh, s);
    const T rn = rsqrt_t(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + s[3] * s[3]);
    s[0] *= rn;
    s[1] *= rn;
    s[2] *= rn;
    s[3] *= rn;
    return true;
  }
  __device__ __forceinline__ bool operator()(const T w[4], uint32_t site, int sg, T s[4]) const {
    const T n2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    if (!(n2 > Tiny<T>::value)) return false;
    const T n = sqrt_t(n2);
    const T alpha = n / temp;
    const T two_pi = (T)6.283185307179586476925286766559;
    T lam2 = -1;
    for (uint32_t att = 0; att < kMaxAttempts; ++att) {
      const U4 r = philox4x32_10(site, sweep, kTagKP | (uint32_t)sg, att, k0, k1);
      const T u0 = unit_open<T>(r.v[0]), u1 = unit_open<T>(r.v[1]);
      const T u2 = unit_open<T>(r.v[2]), u3 = unit_open<T>(r.v[3]);
      const T cs = hb_cos(two_pi * u1);
      const T l2 = -(hb_log(u0) + cs * cs * hb_log(u2)) / (2 * alpha);
      if (u3 * u3 <= 1 - l2) {
        lam2 = l2;
        break;
      }
    }
    if (lam2 < 0) return false;  // attempt cap: subgroup left unchanged
    const U4 d = philox4x32_10(site, sweep, kTagDir | (uint32_t)sg, 0u, k0, k1);
    const T d0 = unit_open<T>(d.v[0]), d1 = unit_open<T>(d.v[1]);
    const T cth = 2 * d0 - 1;
    const T sth = sqrt_t(fmax(T(0), 1 - cth * cth));
    const T phi = two_pi * d1;
    // sqrt(1 - X0^2) = 2 lambda sqrt(1 - lambda^2) for X0 = 1 - 2 lambda^2
    const T rad = 2 * sqrt_t(lam2 * (1 - lam2));
    const T X[4] = {1 - 2 * lam2, rad * sth * hb_cos(phi), rad * sth * hb_sin(phi), rad * cth};
    const T wh[4] = {w[0] / n, w[1] / n, w[2] / n, w[3] / n};
    qmul(X, wh, s);
    // renormalise: keeps repeated low-precision draws on SU(2)
    const T rn = rsqrt_t(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + s[3] * s[3]);
    s[0] *= rn;
    s[1] *= rn;
    s[2] *= rn;
    s[3] *= rn;
    return true;
  }
};

// The draws of a site before its links arrive, shared by its TPS lanes: lane
// r draws subgroups r, r + TPS, ... (the lanes of a wave do this at the same
// time), and the lanes then exchange them, so a lane makes ceil(3 / TPS)
// subgroup draws instead of 3. A lane without a subgroup of its own repeats
// subgroup 2 (kept uniform, unused).
template <int TPS, int SG>
__device__ __forceinline__ void take_draws(HBDraws<float>& d, const float own[6]) {
  constexpr int o = SG % TPS;  // the lane that drew subgroup SG
  d.num[SG] = site_bcast<TPS, o>(own[0]);
  d.u3[SG] = site_bcast<TPS, o>(own[1]);
  d.cth[SG] = site_bcast<TPS, o>(own[2]);
  d.sth[SG] = site_bcast<TPS, o>(own[3]);
  d.cph[SG] = site_bcast<TPS, o>(own[4]);
  d.sph[SG] = site_bcast<TPS, o>(own[5]);
}

template <int TPS>
__device__ __forceinline__ HBDraws<float> split_draws(const UpdHB<float>& u, uint32_t site, int r) {
  constexpr int STEPS = (3 + TPS - 1) / TPS;
  float own[STEPS][6];
#pragma unroll
  for (int k = 0; k < STEPS; ++k) {
    const int sg = k * TPS + r;
    u.draw_one(site, (uint32_t)(sg < 3 ? sg : 2), own[k]);
  }
  HBDraws<float> d;
  take_draws<TPS, 0>(d, own[0]);
  take_draws<TPS, 1>(d, own[1 / TPS]);
  take_draws<TPS, 2>(d, own[2 / TPS]);
  return d;
}

// Gram-Schmidt on rows 0 and 1. A 12-real link rebuilds row 2 =
// conj(row0 x row1), so a norm error of the stored rows reappears, doubled, in
// row 2; a forward update G U mixes row 2 back into rows 0 and 1, and under
// strongly mixing updates (hot annealing) the error grows geometrically.
// Projecting the two stored rows of every forward-updated link keeps it at the
// rounding level (each link is a forward link once per sweep).
template <typename T>
__device__ __forceinline__ void orthonormalize_rows01(Su3<T>& A) {
  T n0 = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) n0 = fma(A.e[0][b].re, A.e[0][b].re, fma(A.e[0][b].im, A.e[0][b].im, n0));
  n0 = rsqrt_t(n0);
#pragma unroll
  for (int b = 0; b < 3; ++b) A.e[0][b] = cx(A.e[0][b].re * n0, A.e[0][b].im * n0);
  Cx<T> ip = cx<T>(0, 0);  // sum conj(row0) row1
#pragma unroll
  for (int b = 0; b < 3; ++b) ip = cmac_cb(ip, A.e[1][b], A.e[0][b]);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const Cx<T> t = cmul(ip, A.e[0][b]);
    A.e[1][b] = csub(A.e[1][b], t);
  }
  T n1 = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) n1 = fma(A.e[1][b].re, A.e[1][b].re, fma(A.e[1][b].im, A.e[1][b].im, n1));
  n1 = rsqrt_t(n1);
#pragma unroll
  for (int b = 0; b < 3; ++b) A.e[1][b] = cx(A.e[1][b].re * n1, A.e[1][b].im * n1);
}

// FP32 rows: the squared norm is summed in FP64 from the FP32 elements (the
// products are exact), and each element moves by x * c with c = 1/|row| - 1
// in one rounding, fmaf(x, c, x). Done wholly in FP32 arithmetic, the
// projection's rounding is not neutral: near unit norm the rounded squared
// norm and the rounded scale factor sit on a grid coarser than the correction
// they carry, so each update moved the link by a small amount that is not a
// gauge transformation and that the next update, which maximises the local
// functional, did not undo; an FP32 12-real field walked off its gauge orbit
// (measured on a 32^4 beta = 6.0 configuration: plaquette +2.4e-5 after
// 10 300 overrelaxation sweeps, against a few 1e-7 either way for the 18-real
// field, which is not projected, and for this form). The sites' g of the
// tracked updates is projected the same way.
__device__ __forceinline__ float unit_scale_minus_one(const Cx<float>* row) {
  double s = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const double x = row[b].re, y = row[b].im;
    s = fma(x, x, fma(y, y, s));
  }
  const double d = s - 1.0;
  double c = d * fma(0.375, d, -0.5);  // (1 + d)^(-1/2) - 1 up to O(d^3)
  if (fabs(d) >= 0x1p-12) c = rsqrt_t(s) - 1.0;
  return (float)c;
}

__device__ __forceinline__ void orthonormalize_rows01(Su3<float>& A) {
  const float c0 = unit_scale_minus_one(A.e[0]);
#pragma unroll
  for (int b = 0; b < 3; ++b)
    A.e[0][b] = cx<float>(fmaf(A.e[0][b].re, c0, A.e[0][b].re), fmaf(A.e[0][b].im, c0, A.e[0][b].im));
  Cx<float> ip = cx<float>(0, 0);  // sum conj(row0) row1
#pragma unroll
  for (int b = 0; b < 3; ++b) ip = cmac_cb(ip, A.e[1][b], A.e[0][b]);
#pragma unroll
  for (int b = 0; b < 3; ++b) A.e[1][b] = csub(A.e[1][b], cmul(ip, A.e[0][b]));
  const float c1 = unit_scale_minus_one(A.e[1]);
#pragma unroll
  for (int b = 0; b < 3; ++b)
    A.e[1][b] = cx<float>(fmaf(A.e[1][b].re, c1, A.e[1][b].re), fmaf(A.e[1][b].im, c1, A.e[1][b].im));
}

// Stochastic relaxation (Sec. 1): per site and subgroup, with probability
// prob the microcanonical step, otherwise overrelaxation with omega (omega = 1:
// relaxation). Draw: Philox key (seed lo, hi), counter (site, sweep,
// 0x1200 | subgroup, 0), first uniform formed in FP64 in every precision, so
// the choice is the same in FP32 and FP64.
constexpr uint32_t kTagSR = 0x1200u;

template <typename T>
struct UpdSR {
  T omega;
  double prob;
  uint32_t k0, k1, sweep;
  __device__ __forceinline__ bool operator()(const T w[4], uint32_t site, int sg, T s[4]) const {
    const U4 d = philox4x32_10(site, sweep, kTagSR | (uint32_t)sg, 0u, k0, k1);
    if (unit_open<double>(d.v[0]) < prob) {
      UpdMicro<T> m;
      return m(w, site, sg, s);
    }
    UpdOR<T> o;
    o.omega = omega;
    return o(w, site, sg, s);
  }
};

template <typename T, class Upd, int I, int J, int SG>
__device__ __forceinline__ void subgroup_step(Su3<T>& K, Su3<T>& G, uint32_t site, const Upd& upd) {
  T w[4], s[4];
  subgroup_w<T, I, J>(K, w);
  if (!upd(w, site, SG, s)) return;
  left_su2<T, I, J>(K, s);
  left_su2<T, I, J>(G, s);
}

// draws a site's update can take before its links arrive: the FP32 heatbath's
// (see HBDraws, split_draws); none for the other updates
struct NoDraws {};
template <int TPS, class Upd>
__device__ __forceinline__ NoDraws pre_draws(const Upd&, uint32_t, int) {
  return {};
}
template <int TPS>
__device__ __forceinline__ HBDraws<float> pre_draws(const UpdHB<float>& u, uint32_t site, int r) {
  return split_draws<TPS>(u, site, r);
}
template <int TPS, typename T, class Upd>
__device__ __forceinline__ bool call_upd(const Upd& u, const T w[4], uint32_t site, int sg, T s[4],
                                         const NoDraws&, int) {
  return u(w, site, sg, s);
}
template <int TPS>
__device__ __forceinline__ bool call_upd(const UpdHB<float>& u, const float w[4], uint32_t site,
                                         int sg, float s[4], const HBDraws<float>& d, int r) {
  return u.template with_draws<TPS>(w, site, sg, s, d, r);
}

// The three subgroup steps with Gtot = G3 G2 G1 built directly: G1 is an
// embedding in rows/cols (0,1), G2 G1 only mixes rows 0 and 2 of it, and
// only the last step is a general row operation. (IEEE arithmetic cannot
// drop the products with the zeros of a unit matrix, so the general form
// would do that work.) A declined step (degenerate subgroup) uses s = 1,
// whose row operation is exact. r is the calling lane's place among its
// site's TPS lanes.
template <typename T, class Upd, int TPS = 1, class D = NoDraws>
__device__ __forceinline__ void build_G(Su3<T>& K, Su3<T>& G, uint32_t site, const Upd& upd,
                                        const D& dr = D(), int r = 0) {
  T w[4], s[4], t[4];
  subgroup_w<T, 0, 1>(K, w);
  if (!call_upd<TPS>(upd, w, site, 0, s, dr, r)) s[0] = 1, s[1] = s[2] = s[3] = 0;
  left_su2<T, 0, 1>(K, s);
  subgroup_w<T, 0, 2>(K, w);
  if (!call_upd<TPS>(upd, w, site, 1, t, dr, r)) t[0] = 1, t[1] = t[2] = t[3] = 0;
  left_su2<T, 0, 2>(K, t);
  // G2 G1: rows of G1 = (g00, g01, 0), (g10, g11, 0), (0, 0, 1)
  const Cx<T> g00 = cx(s[0], s[3]), g01 = cx(s[2], s[1]);
  const Cx<T> g10 = cx(-s[2], s[1]), g11 = cx(s[0], -s[3]);
  const Cx<T> t00 = cx(t[0], t[3]), t02 = cx(t[2], t[1]);
  const Cx<T> t20 = cx(-t[2], t[1]), t22 = cx(t[0], -t[3]);
  G.e[0][0] = cmul(t00, g00);
  G.e[0][1] = cmul(t00, g01);
  G.e[0][2] = t02;
  G.e[1][0] = g10;
  G.e[1][1] = g11;
  G.e[1][2] = cx<T>(0, 0);
  G.e[2][0] = cmul(t20, g00);
  G.e[2][1] = cmul(t20, g01);
  G.e[2][2] = t22;
  subgroup_w<T, 1, 2>(K, w);
  if (call_upd<TPS>(upd, w, site, 2, s, dr, r)) left_su2<T, 1, 2>(G, s);
}

// sum of K over the TPS lanes of one site; every lane ends with the same bits
// (each step adds two partial sums, and addition is commutative)
template <typename T, int TPS>
__device__ __forceinline__ void lane_sum(Su3<T>& K) {
  if (TPS >= 2) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        K.e[a][b].re += quad_xor<1>(K.e[a][b].re);
        K.e[a][b].im += quad_xor<1>(K.e[a][b].im);
      }
  }
  if (TPS >= 4) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        K.e[a][b].re += quad_xor<2>(K.e[a][b].re);
        K.e[a][b].im += quad_xor<2>(K.e[a][b].im);
      }
  }
}

// ---------------------------------------------------------------------------
// half-sweep over the sites of one parity, TPS lanes per site (1, 2 or 4):
// lane r of a site owns the directions mu = r*(4/TPS) ... (r+1)*(4/TPS)-1,
// i.e. their forward links U_mu(x) and backward links U_mu(x-mu). The lanes
// form their partial sums of K, add them across the site's lanes, compute the
// same subgroup transformations, and each updates and stores its own links.
// ---------------------------------------------------------------------------
// TRACK: also accumulate the site transformation into the gauge-transformation
// field Gx (6 complex = rows 0, 1 per site, tiled like the links with one
// direction), g(x) <- Gtot g(x); lane 0
// of the site does it. gid = TPS * h + lane.
// tmask (Coulomb only, may be NULL): one byte per timeslice; the sites of a
// timeslice whose byte is 0 are left alone. Coulomb gauge splits into one
// problem per timeslice (its functional and theta involve spatial links
// only), so a converged timeslice can be frozen while the others go on.
template <typename T, int NC, int GAUGE, class Upd, int TPS, int NT, bool TRACK>
__device__ __forceinline__ void site_half_update(v2<T>* __restrict__ U, const Lat& L,
                                                 const int parity, const Upd& upd,
                                                 v2<T>* __restrict__ Gx, const uint32_t gid,
                                                 const uint8_t* __restrict__ tmask) {
  static_assert(TPS == 1 || TPS == 2 || TPS == 4, "lanes per site");
  constexpr int DPL = 4 / TPS;  // directions per lane
  const uint32_t h = gid / TPS;
  const int r = (int)(gid % TPS);
  if (h >= L.vh) return;  // a site's lanes are all in range or all out
  const Site S = site_of(L, h, parity);
  if constexpr (GAUGE == kCoulomb)
    if (tmask != nullptr && tmask[S.t] == 0) return;  // all lanes of the site agree
  uint32_t hb[DPL];
  Su3<T> Uf[DPL], Ub[DPL];
#pragma unroll
  for (int d = 0; d < DPL; ++d) {
    const int mu = r * DPL + d;
    hb[d] = back_h(L, h, S, mu);
    load_link<T, NC, NT>(U + link_offset<NC>(L.vp, parity, mu, h), Uf[d]);
    load_link<T, NC, NT>(U + link_offset<NC>(L.vp, 1 - parity, mu, hb[d]), Ub[d]);
  }
  const uint32_t site = 2 * h + S.xodd;
  const auto dr = pre_draws<TPS>(upd, site, r);  // while the loads are in flight
  Su3<T> K;
  set_zero(K);
#pragma unroll
  for (int d = 0; d < DPL; ++d) {
    const int mu = r * DPL + d;
    if (TPS == 1 && mu < FirstDir<GAUGE>::value) continue;
    const T on = (mu >= FirstDir<GAUGE>::value) ? T(1) : T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const Cx<T> v = cadd(Uf[d].e[a][b], cconj(Ub[d].e[b][a]));
        if (TPS == 1)
          K.e[a][b] = cadd(K.e[a][b], v);
        else
          K.e[a][b] = cx(fma(on, v.re, K.e[a][b].re), fma(on, v.im, K.e[a][b].im));
      }
  }
  lane_sum<T, TPS>(K);
  Su3<T> G;
  build_G<T, Upd, TPS>(K, G, site, upd, dr, r);
  if (TRACK && r == 0) {
    v2<T>* gp = Gx + link_offset<6, 1>(L.vp, parity, 0, h);
    Su3<T> gx, A;
    load_link<T, 6, NT>(gp, gx);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Cx<T> f = cmul(G.e[a][0], gx.e[0][b]);
        f = cmac(f, G.e[a][1], gx.e[1][b]);
        A.e[a][b] = cmac(f, G.e[a][2], gx.e[2][b]);
      }
    orthonormalize_rows01(A);  // g is stored as 12 reals and left-multiplied too
    store_link<T, 6, NT>(gp, A);
  }
  constexpr int R = NC / 3;  // stored rows
#pragma unroll
  for (int d = 0; d < DPL; ++d) {
    const int mu = r * DPL + d;
    Su3<T> A;
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Cx<T> f = cmul(G.e[a][0], Uf[d].e[0][b]);
        f = cmac(f, G.e[a][1], Uf[d].e[1][b]);
        A.e[a][b] = cmac(f, G.e[a][2], Uf[d].e[2][b]);
      }
    if (NC == 6) orthonormalize_rows01(A);
    store_link<T, NC, NT>(U + link_offset<NC>(L.vp, parity, mu, h), A);
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Cx<T> f = cx<T>(0, 0);
        f = cmac_cb(f, Ub[d].e[a][0], G.e[b][0]);
        f = cmac_cb(f, Ub[d].e[a][1], G.e[b][1]);
        A.e[a][b] = cmac_cb(f, Ub[d].e[a][2], G.e[b][2]);
      }
    store_link<T, NC, NT>(U + link_offset<NC>(L.vp, 1 - parity, mu, hb[d]), A);
  }
}

// Half-sweeps alternate their direction through the field: RED walks the
// blocks upwards, BLACK downwards. Each half-sweep then begins on the part of
// the field the previous one touched last, which the 256 MB Infinity Cache
// still holds, instead of on the part it evicted longest ago. The sites of
// one parity are independent, so the order changes no result.
__device__ __forceinline__ uint32_t sweep_block(const int parity) {
  return parity ? gridDim.x - 1 - blockIdx.x : blockIdx.x;
}

// occupancy request (minimum waves per SIMD) of the sweep kernels: FP64 with
// 4 lanes per site fits 3 waves (<= 168 registers)
template <typename T, int TPS>
struct SweepWaves {
  static constexpr int value = 1;
};

template <typename T, int NC, int GAUGE, class Upd, int TPS, int NT, bool TRACK = false>
__global__ __launch_bounds__(kBlock, (SweepWaves<T, TPS>::value)) void k_update_half(v2<T>* __restrict__ U, const Lat L,
                                                        const int parity, const Upd upd,
                                                        v2<T>* __restrict__ Gx = nullptr,
                                                        const uint8_t* __restrict__ tmask = nullptr) {
  site_half_update<T, NC, GAUGE, Upd, TPS, NT, TRACK>(U, L, parity, upd, Gx,
                                                      sweep_block(parity) * kBlock + threadIdx.x,
                                                      tmask);
}

// ---------------------------------------------------------------------------
// maximally Abelian gauge: maximise R = sum_{x,mu} sum_k |U_mu(x)_kk|^2 (the
// gauge named in Sec. 1; functional from the literature). Under G = embed(a)
// on the subgroup (i, j) the diagonal entries of the site's links that change
// are linear in the quaternion a = (a0, a1, a2, a3):
//   (G U)_ii   = U_ii a0 + i U_ji a1 + U_ji a2 + i U_ii a3
//   (G U)_jj   = U_jj a0 + i U_ij a1 - U_ij a2 - i U_jj a3
//   (W G^+)_ii = W_ii a0 - i W_ij a1 + W_ij a2 - i W_ii a3
//   (W G^+)_jj = W_jj a0 - i W_ji a1 - W_ji a2 + i W_jj a3
// (U forward, W backward links), so the site's R is a^T M a + const with
// M_kl = sum Re(c_k conj(c_l)) over these coefficient vectors c. The diagonal
// phases of the subgroup (rotating (a0, a3) and (a1, a2) together) leave R
// unchanged, so the maximiser is taken with a3 = 0: the top eigenvector of
// the 3x3 block of M on (a0, a1, a2), with a0 >= 0.
// ---------------------------------------------------------------------------
// M block entries m = (M00, M01, M02, M11, M12, M22) += Re(c_k conj(c_l))
template <typename T>
__device__ __forceinline__ void mag_acc(T m[6], const Cx<T>& c0, const Cx<T>& c1,
                                        const Cx<T>& c2) {
  m[0] = fma(c0.re, c0.re, fma(c0.im, c0.im, m[0]));
  m[1] = fma(c0.re, c1.re, fma(c0.im, c1.im, m[1]));
  m[2] = fma(c0.re, c2.re, fma(c0.im, c2.im, m[2]));
  m[3] = fma(c1.re, c1.re, fma(c1.im, c1.im, m[3]));
  m[4] = fma(c1.re, c2.re, fma(c1.im, c2.im, m[4]));
  m[5] = fma(c2.re, c2.re, fma(c2.im, c2.im, m[5]));
}
template <typename T>
__device__ __forceinline__ Cx<T> times_i(const Cx<T>& z) { return cx<T>(-z.im, z.re); }
template <typename T>
__device__ __forceinline__ Cx<T> times_mi(const Cx<T>& z) { return cx<T>(z.im, -z.re); }
template <typename T>
__device__ __forceinline__ Cx<T> neg(const Cx<T>& z) { return cx<T>(-z.re, -z.im); }

template <typename T>
__device__ __forceinline__ void mag_forward(T m[6], const Su3<T>& U, int i, int j) {
  mag_acc(m, U.e[i][i], times_i(U.e[j][i]), U.e[j][i]);
  mag_acc(m, U.e[j][j], times_i(U.e[i][j]), neg(U.e[i][j]));
}
template <typename T>
__device__ __forceinline__ void mag_backward(T m[6], const Su3<T>& W, int i, int j) {
  mag_acc(m, W.e[i][i], times_mi(W.e[i][j]), W.e[i][j]);
  mag_acc(m, W.e[j][j], times_mi(W.e[j][i]), neg(W.e[j][i]));
}

template <typename T>
struct JacobiTol;
template <>
struct JacobiTol<float> {
  static constexpr float value = 1e-14f;  // off-diagonal^2 relative to diagonal^2
};
template <>
struct JacobiTol<double> {
  static constexpr double value = 1e-34;
};

// top eigenvector of the symmetric 3x3 m = (M00, M01, M02, M11, M12, M22) by
// cyclic Jacobi rotations (Golub & Van Loan, Sec. 8.5), at most 6 sweeps,
// stopping when the off-diagonal part is at rounding level; unit length,
// a0 >= 0 (then a1, a2 >= 0). Returns false if m vanishes.
template <typename T>
__device__ __forceinline__ bool mag_top_eigvec(const T m[6], T v[3]) {
  T A[3][3] = {{m[0], m[1], m[2]}, {m[1], m[3], m[4]}, {m[2], m[4], m[5]}};
  T Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  const T nrm = fabs(m[0]) + fabs(m[3]) + fabs(m[5]) + 2 * (fabs(m[1]) + fabs(m[2]) + fabs(m[4]));
  if (!(nrm > Tiny<T>::value)) return false;
  for (int sw = 0; sw < 6; ++sw) {
    const T off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const T dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= JacobiTol<T>::value * dia) break;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == T(0)) continue;
        const T theta = (A[q][q] - A[p][p]) / (T(2) * A[p][q]);
        const T t = (theta >= T(0) ? T(1) : T(-1)) / (fabs(theta) + sqrt(theta * theta + T(1)));
        const T c = T(1) / sqrt(t * t + T(1)), sn = t * c;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T qkp = Q[k][p], qkq = Q[k][q];
          Q[k][p] = c * qkp - sn * qkq;
          Q[k][q] = sn * qkp + c * qkq;
        }
      }
  }
  int best = 0;
  T lb = A[0][0];
  if (A[1][1] > lb) {
    best = 1;
    lb = A[1][1];
  }
  if (A[2][2] > lb) best = 2;
  T x = Q[0][0], y = Q[1][0], z = Q[2][0];
  if (best == 1) {
    x = Q[0][1];
    y = Q[1][1];
    z = Q[2][1];
  } else if (best == 2) {
    x = Q[0][2];
    y = Q[1][2];
    z = Q[2][2];
  }
  const bool flip = x < T(0) || (x == T(0) && (y < T(0) || (y == T(0) && z < T(0))));
  const T r = (flip ? T(-1) : T(1)) / sqrt(x * x + y * y + z * z);
  v[0] = x * r;
  v[1] = y * r;
  v[2] = z * r;
  return true;
}

// MAG half-sweep (Alg. 1 with the MAG local step), TPS lanes per site as in
// site_half_update: for each subgroup in turn the lanes add their parts of M,
// every lane finds the same maximiser and its power (Upd: g^omega from the
// unit quaternion), and each lane transforms its own links in registers,
// since M of the next subgroup depends on the updated links quadratically.
template <typename T, int NC, class Upd, int TPS, int NT, bool TRACK>
__device__ __forceinline__ void site_mag_update(v2<T>* __restrict__ U, const Lat& L,
                                                const int parity, const Upd& upd,
                                                v2<T>* __restrict__ Gx, const uint32_t gid) {
  static_assert(TPS == 1 || TPS == 2 || TPS == 4, "lanes per site");
  constexpr int DPL = 4 / TPS;
  const uint32_t h = gid / TPS;
  const int r = (int)(gid % TPS);
  if (h >= L.vh) return;  // a site's lanes are all in range or all out
  const Site S = site_of(L, h, parity);
  uint32_t hb[DPL];
  Su3<T> Uf[DPL], Ub[DPL];
#pragma unroll
  for (int d = 0; d < DPL; ++d) {
    const int mu = r * DPL + d;
    hb[d] = back_h(L, h, S, mu);
    load_link<T, NC, NT>(U + link_offset<NC>(L.vp, parity, mu, h), Uf[d]);
    load_link<T, NC, NT>(U + link_offset<NC>(L.vp, 1 - parity, mu, hb[d]), Ub[d]);
  }
  Su3<T> Gt;
  if (TRACK) set_unit(Gt);
  const uint32_t site = 2 * h + S.xodd;
#pragma unroll
  for (int sg = 0; sg < 3; ++sg) {
    const int i = sg == 2 ? 1 : 0, j = sg == 0 ? 1 : 2;
    T m[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < DPL; ++d) {
      mag_forward(m, Uf[d], i, j);
      mag_backward(m, Ub[d], i, j);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      if (TPS >= 2) m[k] += quad_xor<1>(m[k]);
      if (TPS >= 4) m[k] += quad_xor<2>(m[k]);
    }
    T v[3];
    if (!mag_top_eigvec(m, v)) continue;
    const T w[4] = {v[0], v[1], v[2], T(0)};
    T q[4];
    if (!upd(w, site, sg, q)) continue;
    // SU(2) block [[q0 + i q3, q2 + i q1], [-q2 + i q1, q0 - i q3]] on (i, j)
    const Cx<T> g00 = cx<T>(q[0], q[3]), g01 = cx<T>(q[2], q[1]);
    const Cx<T> g10 = cx<T>(-q[2], q[1]), g11 = cx<T>(q[0], -q[3]);
#pragma unroll
    for (int d = 0; d < DPL; ++d) {
#pragma unroll
      for (int b = 0; b < 3; ++b) {  // rows i, j of G U
        const Cx<T> ui = Uf[d].e[i][b], uj = Uf[d].e[j][b];
        Uf[d].e[i][b] = cmac(cmul(g00, ui), g01, uj);
        Uf[d].e[j][b] = cmac(cmul(g10, ui), g11, uj);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {  // columns i, j of W G^+
        const Cx<T> wi = Ub[d].e[a][i], wj = Ub[d].e[a][j];
        Ub[d].e[a][i] = cmac_cb(cmac_cb(cx<T>(0, 0), wi, g00), wj, g01);
        Ub[d].e[a][j] = cmac_cb(cmac_cb(cx<T>(0, 0), wi, g10), wj, g11);
      }
    }
    if (TRACK) {
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const Cx<T> gi = Gt.e[i][b], gj = Gt.e[j][b];
        Gt.e[i][b] = cmac(cmul(g00, gi), g01, gj);
        Gt.e[j][b] = cmac(cmul(g10, gi), g11, gj);
      }
    }
  }
  if (TRACK && r == 0) {
    v2<T>* gp = Gx + link_offset<6, 1>(L.vp, parity, 0, h);
    Su3<T> gx, A;
    load_link<T, 6, NT>(gp, gx);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Cx<T> f = cmul(Gt.e[a][0], gx.e[0][b]);
        f = cmac(f, Gt.e[a][1], gx.e[1][b]);
        A.e[a][b] = cmac(f, Gt.e[a][2], gx.e[2][b]);
      }
    orthonormalize_rows01(A);
    store_link<T, 6, NT>(gp, A);
  }
#pragma unroll
  for (int d = 0; d < DPL; ++d) {
    const int mu = r * DPL + d;
    if (NC == 6) orthonormalize_rows01(Uf[d]);
    store_link<T, NC, NT>(U + link_offset<NC>(L.vp, parity, mu, h), Uf[d]);
    store_link<T, NC, NT>(U + link_offset<NC>(L.vp, 1 - parity, mu, hb[d]), Ub[d]);
  }
}

// occupancy request of the MAG kernels: FP64 with 2 lanes per site needs a
// few registers more than two waves per SIMD allow (the 2048-site tiles put
// the link components 32 KB apart, beyond the loads' immediate offsets, so
// each component needs its own address); two waves with a few registers
// spilled beat one wave
template <typename T, int TPS>
struct MagWaves {
  static constexpr int value = (sizeof(T) == 8 && TPS == 2) ? 2 : 1;
};

template <typename T, int NC, class Upd, int TPS, int NT, bool TRACK = false>
__global__ __launch_bounds__(kBlock, (MagWaves<T, TPS>::value)) void k_mag_half(v2<T>* __restrict__ U, const Lat L,
                                                     const int parity, const Upd upd,
                                                     v2<T>* __restrict__ Gx = nullptr) {
  site_mag_update<T, NC, Upd, TPS, NT, TRACK>(U, L, parity, upd, Gx,
                                              sweep_block(parity) * kBlock + threadIdx.x);
}

// ---------------------------------------------------------------------------
// batches of independent lattices (Gribov copies, uneven extents): one launch
// covers the lattices of a table, entry k owning the blocks
// [first_block[k], first_block[k+1]), and map[b] names the entry of block b
// (one load per block instead of a search of the table); the host rebuilds
// table and map without the lattices that have left the phase, so a launch
// covers active lattices only.
// ---------------------------------------------------------------------------
template <typename T>
struct BatchEntry {
  Lat L;
  v2<T>* U;   // the lattice's device field
  v2<T>* Gx;  // its gauge-transformation field (tracked runs) or null
  uint32_t first_block;
  uint32_t index;  // lattice number (keys the annealing draws)
};

// per-lattice update policy: the annealing draws of lattice l use the key
// seed + l, so that a batched lattice draws what a run of it alone with that
// seed draws
template <class Upd>
__device__ __forceinline__ Upd for_lattice(const Upd& u, uint32_t) {
  return u;
}
template <typename T>
__device__ __forceinline__ UpdHB<T> for_lattice(const UpdHB<T>& u, uint32_t l) {
  UpdHB<T> v = u;
  const uint64_t seed = (((uint64_t)u.k1 << 32) | u.k0) + l;
  v.k0 = (uint32_t)seed;
  v.k1 = (uint32_t)(seed >> 32);
  return v;
}
template <typename T>
__device__ __forceinline__ UpdSR<T> for_lattice(const UpdSR<T>& u, uint32_t l) {
  UpdSR<T> v = u;
  const uint64_t seed = (((uint64_t)u.k1 << 32) | u.k0) + l;
  v.k0 = (uint32_t)seed;
  v.k1 = (uint32_t)(seed >> 32);
  return v;
}

template <typename T, int NC, class Upd, int TPS, int NT, bool TRACK>
__global__ __launch_bounds__(kBlock) void k_update_half_batch(const BatchEntry<T>* __restrict__ tab,
                                                              const uint32_t* __restrict__ map,
                                                              const int parity, const Upd upd) {
  const uint32_t blk = sweep_block(parity);
  const BatchEntry<T> e = tab[map[blk]];
  site_half_update<T, NC, kLandau, Upd, TPS, NT, TRACK>(
      e.U, e.L, parity, for_lattice(upd, e.index), e.Gx,
      (blk - e.first_block) * kBlock + threadIdx.x, nullptr);
}

// ---------------------------------------------------------------------------
// reductions (FP64 accumulation, fixed order: wave shuffle, LDS, per-block
// partials, then one finishing block per output)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// sum over the block (kBlock threads); result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kBlock / 64; ++k) r += lds[k];
  __syncthreads();
  return r;
}

template <typename T, int NC>
__device__ __forceinline__ void load_link_f64(const v2<T>* __restrict__ q, Su3<double>& A) {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const v2<T> v = q[c * kTile];
    A.e[c / 3][c % 3] = cx<double>((double)v.x, (double)v.y);
  }
  if (NC == 6) rebuild_row2(A);
}

// grid (blocks per timeslice, nt); thread -> half index within timeslice t,
// both parities. partial[(t*bpt + bx)*2 + {0: F, 1: theta}]
template <typename T, int NC, int GAUGE>
__global__ __launch_bounds__(kBlock) void k_measure(const v2<T>* __restrict__ U, const Lat L,
                                                    double* __restrict__ partial) {
  __shared__ double lds[kBlock / 64];
  const uint32_t t = blockIdx.y;
  const uint32_t ht = blockIdx.x * kBlock + threadIdx.x;
  double f = 0, th = 0;
  if (ht < L.st) {
    const uint32_t h = t * L.st + ht;
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
      const Site S = site_of(L, h, p);
      Su3<double> K;
      set_zero(K);
#pragma unroll 1
      for (int mu = FirstDir<GAUGE>::value; mu < 4; ++mu) {
        Su3<double> A, B;
        load_link_f64<T, NC>(U + link_offset<NC>(L.vp, p, mu, h), A);
        load_link_f64<T, NC>(U + link_offset<NC>(L.vp, 1 - p, mu, back_h(L, h, S, mu)), B);
        f += A.e[0][0].re + A.e[1][1].re + A.e[2][2].re;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b)
            K.e[a][b] = cadd(K.e[a][b], cadd(A.e[a][b], cconj(B.e[b][a])));
      }
      // Delta = traceless part of (K - K^dag)/(2i); theta density tr[Delta Delta^dag]
      const double d0 = K.e[0][0].im, d1 = K.e[1][1].im, d2 = K.e[2][2].im;
      const double tr3 = (d0 + d1 + d2) / 3.0;
      double acc = (d0 - tr3) * (d0 - tr3) + (d1 - tr3) * (d1 - tr3) + (d2 - tr3) * (d2 - tr3);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          if (a == b) continue;
          const Cx<double> z = csub(K.e[a][b], cconj(K.e[b][a]));
          acc += 0.25 * (z.re * z.re + z.im * z.im);
        }
      th += acc;
    }
  }
  f = block_sum(f, lds);
  th = block_sum(th, lds);
  if (threadIdx.x == 0) {
    const size_t o = ((size_t)t * gridDim.x + blockIdx.x) * 2;
    partial[o] = f;
    partial[o + 1] = th;
  }
}

// MAG measurement, same grid and partials as k_measure: F part = sum over
// the forward links of sum_k |U_kk|^2, theta part = sum over the subgroups of
// M01^2 + M02^2 (the derivatives of R along the off-diagonal generators are
// 2 M01, 2 M02 at the identity), with M from the 8 links of the site.
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_measure_mag(const v2<T>* __restrict__ U, const Lat L,
                                                        double* __restrict__ partial) {
  __shared__ double lds[kBlock / 64];
  const uint32_t t = blockIdx.y;
  const uint32_t ht = blockIdx.x * kBlock + threadIdx.x;
  double f = 0, th = 0;
  if (ht < L.st) {
    const uint32_t h = t * L.st + ht;
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
      const Site S = site_of(L, h, p);
      double m[3][6] = {};
#pragma unroll 1
      for (int mu = 0; mu < 4; ++mu) {
        Su3<double> A, B;
        load_link_f64<T, NC>(U + link_offset<NC>(L.vp, p, mu, h), A);
        load_link_f64<T, NC>(U + link_offset<NC>(L.vp, 1 - p, mu, back_h(L, h, S, mu)), B);
#pragma unroll
        for (int k = 0; k < 3; ++k)
          f += A.e[k][k].re * A.e[k][k].re + A.e[k][k].im * A.e[k][k].im;
#pragma unroll
        for (int sg = 0; sg < 3; ++sg) {
          const int i = sg == 2 ? 1 : 0, j = sg == 0 ? 1 : 2;
          mag_forward(m[sg], A, i, j);
          mag_backward(m[sg], B, i, j);
        }
      }
#pragma unroll
      for (int sg = 0; sg < 3; ++sg) th += m[sg][1] * m[sg][1] + m[sg][2] * m[sg][2];
    }
  }
  f = block_sum(f, lds);
  th = block_sum(th, lds);
  if (threadIdx.x == 0) {
    const size_t o = ((size_t)t * gridDim.x + blockIdx.x) * 2;
    partial[o] = f;
    partial[o + 1] = th;
  }
}

// batched Landau measurement: thread = half index of one lattice, both
// parities; lattice l owns blocks [first_block[l], first_block[l+1]);
// partial[2*block + {0: F, 1: theta}]
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_measure_batch(const BatchEntry<T>* __restrict__ tab,
                                                          const uint32_t* __restrict__ map,
                                                          double* __restrict__ partial) {
  __shared__ double lds[kBlock / 64];
  const BatchEntry<T> e = tab[map[blockIdx.x]];
  const Lat& L = e.L;
  const uint32_t h = (blockIdx.x - e.first_block) * kBlock + threadIdx.x;
  double f = 0, th = 0;
  if (h < L.vh) {
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
      const Site S = site_of(L, h, p);
      Su3<double> K;
      set_zero(K);
#pragma unroll 1
      for (int mu = 0; mu < 4; ++mu) {
        Su3<double> A, B;
        load_link_f64<T, NC>(e.U + link_offset<NC>(L.vp, p, mu, h), A);
        load_link_f64<T, NC>(e.U + link_offset<NC>(L.vp, 1 - p, mu, back_h(L, h, S, mu)), B);
        f += A.e[0][0].re + A.e[1][1].re + A.e[2][2].re;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b)
            K.e[a][b] = cadd(K.e[a][b], cadd(A.e[a][b], cconj(B.e[b][a])));
      }
      const double d0 = K.e[0][0].im, d1 = K.e[1][1].im, d2 = K.e[2][2].im;
      const double tr3 = (d0 + d1 + d2) / 3.0;
      double acc = (d0 - tr3) * (d0 - tr3) + (d1 - tr3) * (d1 - tr3) + (d2 - tr3) * (d2 - tr3);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          if (a == b) continue;
          const Cx<double> z = csub(K.e[a][b], cconj(K.e[b][a]));
          acc += 0.25 * (z.re * z.re + z.im * z.im);
        }
      th += acc;
    }
  }
  f = block_sum(f, lds);
  th = block_sum(th, lds);
  if (threadIdx.x == 0) {
    partial[2 * (size_t)blockIdx.x] = f;
    partial[2 * (size_t)blockIdx.x + 1] = th;
  }
}

// one block per table entry k: F[l] = sum / (12 V_l), theta[l] = sum / (3 V_l)
// over the entry's blocks, l = its lattice number
template <typename T>
__global__ __launch_bounds__(kBlock) void k_finish_batch(const BatchEntry<T>* __restrict__ tab,
                                                         const int n, const uint32_t total_blocks,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ F,
                                                         double* __restrict__ th) {
  __shared__ double lds[kBlock / 64];
  const int k = blockIdx.x;
  const uint32_t b0 = tab[k].first_block;
  const uint32_t b1 = (k + 1 < n) ? tab[k + 1].first_block : total_blocks;
  double a = 0, b = 0;
  for (uint32_t k = b0 + threadIdx.x; k < b1; k += kBlock) {
    a += partial[2 * (size_t)k];
    b += partial[2 * (size_t)k + 1];
  }
  a = block_sum(a, lds);
  b = block_sum(b, lds);
  if (threadIdx.x == 0) {
    const double V = 2.0 * tab[k].L.vh;
    F[tab[k].index] = a / (12.0 * V);
    th[tab[k].index] = b / (3.0 * V);
  }
}

// one block per output group: sums n_per partial pairs starting at group*n_per
static __global__ __launch_bounds__(kBlock) void k_finish(const double* __restrict__ partial,
                                                   uint32_t n_per, double norm0, double norm1,
                                                   double* __restrict__ out0,
                                                   double* __restrict__ out1) {
  __shared__ double lds[kBlock / 64];
  const size_t base = (size_t)blockIdx.x * n_per;
  double a = 0, b = 0;
  for (uint32_t k = threadIdx.x; k < n_per; k += kBlock) {
    a += partial[(base + k) * 2];
    b += partial[(base + k) * 2 + 1];
  }
  a = block_sum(a, lds);
  b = block_sum(b, lds);
  if (threadIdx.x == 0) {
    if (out0) out0[blockIdx.x] = a / norm0;
    if (out1) out1[blockIdx.x] = b / norm1;
  }
}

// average plaquette: partial[(bx)*2 + {0: sum Re tr U_P / 3, 1: 0}]
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_plaquette(const v2<T>* __restrict__ U, const Lat L,
                                                      double* __restrict__ partial) {
  __shared__ double lds[kBlock / 64];
  const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
  double acc = 0;
  if (h < L.vh) {
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
      const Site S = site_of(L, h, p);
#pragma unroll 1
      for (int mu = 0; mu < 4; ++mu)
#pragma unroll 1
        for (int nu = mu + 1; nu < 4; ++nu) {
          Su3<double> A, B, C, D;
          load_link_f64<T, NC>(U + link_offset<NC>(L.vp, p, mu, h), A);
          load_link_f64<T, NC>(U + link_offset<NC>(L.vp, 1 - p, nu, fwd_h(L, h, S, mu)), B);
          load_link_f64<T, NC>(U + link_offset<NC>(L.vp, 1 - p, mu, fwd_h(L, h, S, nu)), C);
          load_link_f64<T, NC>(U + link_offset<NC>(L.vp, p, nu, h), D);
          // Re tr[A B C^dag D^dag] = Re sum_{a,b} (A B)_{ab} (D C)^*_{ab}
          double tr = 0;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              Cx<double> ab = cx<double>(0, 0), dc = cx<double>(0, 0);
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                ab = cmac(ab, A.e[a][k], B.e[k][b]);
                dc = cmac(dc, D.e[a][k], C.e[k][b]);
              }
              tr += ab.re * dc.re + ab.im * dc.im;
            }
          acc += tr / 3.0;
        }
    }
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) {
    partial[(size_t)blockIdx.x * 2] = acc;
    partial[(size_t)blockIdx.x * 2 + 1] = 0;
  }
}

// ---------------------------------------------------------------------------
// layout conversion
// ---------------------------------------------------------------------------
// Gram-Schmidt in FP64 on rows 0, 1, then row 2 = conj(row0 x row1)
__device__ __forceinline__ void gram_schmidt(Su3<double>& A) {
  double n0 = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) n0 += A.e[0][b].re * A.e[0][b].re + A.e[0][b].im * A.e[0][b].im;
  n0 = 1.0 / sqrt(n0);
#pragma unroll
  for (int b = 0; b < 3; ++b) A.e[0][b] = cx(A.e[0][b].re * n0, A.e[0][b].im * n0);
  Cx<double> ip = cx<double>(0, 0);  // sum conj(row0) row1
#pragma unroll
  for (int b = 0; b < 3; ++b) ip = cmac_cb(ip, A.e[1][b], A.e[0][b]);
#pragma unroll
  for (int b = 0; b < 3; ++b) A.e[1][b] = csub(A.e[1][b], cmul(ip, A.e[0][b]));
  double n1 = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) n1 += A.e[1][b].re * A.e[1][b].re + A.e[1][b].im * A.e[1][b].im;
  n1 = 1.0 / sqrt(n1);
#pragma unroll
  for (int b = 0; b < 3; ++b) A.e[1][b] = cx(A.e[1][b].re * n1, A.e[1][b].im * n1);
  rebuild_row2(A);
}

template <typename Td, int NCd>
__device__ __forceinline__ void store_link_from_f64(v2<Td>* __restrict__ q,
                                                    const Su3<double>& A) {
#pragma unroll
  for (int c = 0; c < NCd; ++c) {
    v2<Td> v;
    v.x = (Td)A.e[c / 3][c % 3].re;
    v.y = (Td)A.e[c / 3][c % 3].im;
    q[c * kTile] = v;
  }
}

// grid (ceil(vh/kBlock), 8): blockIdx.y = p*4 + mu; vp = padded block stride
template <typename Ts, int NCs, typename Td, int NCd>
__global__ __launch_bounds__(kBlock) void k_convert(const v2<Ts>* __restrict__ src,
                                                    v2<Td>* __restrict__ dst, const uint32_t vh,
                                                    const uint32_t vp, const int reunit) {
  const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
  if (h >= vh) return;
  const int p = blockIdx.y >> 2, mu = blockIdx.y & 3;
  Su3<double> A;
  load_link_f64<Ts, NCs>(src + link_offset<NCs>(vp, p, mu, h), A);
  if (reunit) gram_schmidt(A);
  store_link_from_f64<Td, NCd>(dst + link_offset<NCd>(vp, p, mu, h), A);
}

// in place: same buffer, each thread reads and then writes its own link
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_reunitarize(v2<T>* U, const uint32_t vh,
                                                       const uint32_t vp) {
  const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
  if (h >= vh) return;
  v2<T>* q = U + link_offset<NC>(vp, blockIdx.y >> 2, blockIdx.y & 3, h);
  Su3<double> A;
  load_link_f64<T, NC>(q, A);
  gram_schmidt(A);
  store_link_from_f64<T, NC>(q, A);
}

// canonical complex128 U[s][mu][3][3] -> device layout; grid (ceil(V/kBlock), 4)
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_pack(const double* __restrict__ src,
                                                 v2<T>* __restrict__ dst, const Lat L) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= 2 * L.vh) return;
  const int mu = blockIdx.y;
  const uint32_t h = s >> 1;
  const Site S = site_of(L, h, 0);
  const int p = (int)((S.t + S.z + S.y + (s & 1u)) & 1u);
  const double* q = src + ((size_t)s * 4 + mu) * 18;
  v2<T>* d = dst + link_offset<NC>(L.vp, p, mu, h);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    v2<T> v;
    v.x = (T)q[2 * c];
    v.y = (T)q[2 * c + 1];
    d[c * kTile] = v;
  }
}

template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_unpack(const v2<T>* __restrict__ src,
                                                   double* __restrict__ dst, const Lat L) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= 2 * L.vh) return;
  const int mu = blockIdx.y;
  const uint32_t h = s >> 1;
  const Site S = site_of(L, h, 0);
  const int p = (int)((S.t + S.z + S.y + (s & 1u)) & 1u);
  Su3<double> A;
  load_link_f64<T, NC>(src + link_offset<NC>(L.vp, p, mu, h), A);
  double* q = dst + ((size_t)s * 4 + mu) * 18;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    q[2 * c] = A.e[c / 3][c % 3].re;
    q[2 * c + 1] = A.e[c / 3][c % 3].im;
  }
}

// canonical complex128 g[s][3][3] -> gauge-transformation field (rows 0 and
// 1, rounded to Tg); grid ceil(V/kBlock)
template <typename Tg>
__global__ __launch_bounds__(kBlock) void k_pack_gauge(const double* __restrict__ src,
                                                       v2<Tg>* __restrict__ G, const Lat L) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= 2 * L.vh) return;
  const uint32_t h = s >> 1;
  const Site S = site_of(L, h, 0);
  const int p = (int)((S.t + S.z + S.y + (s & 1u)) & 1u);
  const double* q = src + (size_t)s * 18;
  v2<Tg>* d = G + link_offset<6, 1>(L.vp, p, 0, h);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    v2<Tg> v;
    v.x = (Tg)q[2 * c];
    v.y = (Tg)q[2 * c + 1];
    d[c * kTile] = v;
  }
}

// gauge-transformation field (rows 0 and 1 of g, ND = 1) -> canonical
// complex128 g[s][3][3], row 2 rebuilt in FP64; grid ceil(V/kBlock)
template <typename Tg>
__global__ __launch_bounds__(kBlock) void k_unpack_gauge(const v2<Tg>* __restrict__ G,
                                                         double* __restrict__ dst, const Lat L) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= 2 * L.vh) return;
  const uint32_t h = s >> 1;
  const Site S = site_of(L, h, 0);
  const int p = (int)((S.t + S.z + S.y + (s & 1u)) & 1u);
  Su3<double> A;
  load_link_f64<Tg, 6>(G + link_offset<6, 1>(L.vp, p, 0, h), A);
  double* q = dst + (size_t)s * 18;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    q[2 * c] = A.e[c / 3][c % 3].re;
    q[2 * c + 1] = A.e[c / 3][c % 3].im;
  }
}

// the unit field in the device layout (scratch fields of the autotuner, the
// gauge-transformation field of the mixed-precision driver, ND = 1); grid.y =
// 2 * ND (parity, direction), padding sites included (grid.x covers vp)
template <typename T, int NC, int ND>
__global__ __launch_bounds__(kBlock) void k_fill_unit(v2<T>* __restrict__ U, const uint32_t vp) {
  const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
  if (h >= vp) return;
  v2<T>* q = U + link_offset<NC, ND>(vp, blockIdx.y / ND, blockIdx.y % ND, h);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    v2<T> v;
    v.x = (c % 4 == 0) ? T(1) : T(0);  // c = 0, 4, 8 are the diagonal
    v.y = 0;
    q[c * kTile] = v;
  }
}

// batched in-place reunitarisation of the lattices of a table (8 link blocks each)
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_reunitarize_batch(const BatchEntry<T>* __restrict__ tab,
                                                              const uint32_t* __restrict__ map) {
  const BatchEntry<T> e = tab[map[blockIdx.x]];
  const uint32_t h = (blockIdx.x - e.first_block) * kBlock + threadIdx.x;
  if (h >= e.L.vh) return;
#pragma unroll 1
  for (int pm = 0; pm < 8; ++pm) {
    Su3<double> A;
    v2<T>* q = e.U + link_offset<NC>(e.L.vp, pm >> 2, pm & 3, h);
    load_link_f64<T, NC>(q, A);
    gram_schmidt(A);
    store_link_from_f64<T, NC>(q, A);
  }
}

// U_mu(x) <- g(x) U_mu(x) g(x+mu)^dag in FP64, with g (Tg, rows 0 and 1, one
// tiled block per parity) projected onto SU(3) by Gram-Schmidt first. Each
// thread owns the four forward links of one site and only reads g, so the
// update is in place. grid (ceil(vh/kBlock), 2): blockIdx.y = parity.
template <typename T, int NC, typename Tg>
__global__ __launch_bounds__(kBlock) void k_apply_gauge(v2<T>* __restrict__ U,
                                                        const v2<Tg>* __restrict__ Gx, const Lat L) {
  const uint32_t h = blockIdx.x * kBlock + threadIdx.x;
  if (h >= L.vh) return;
  const int p = blockIdx.y;
  const Site S = site_of(L, h, p);
  Su3<double> g;
  load_link_f64<Tg, 6>(Gx + link_offset<6, 1>(L.vp, p, 0, h), g);
  gram_schmidt(g);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    Su3<double> gn, A, B;
    load_link_f64<Tg, 6>(Gx + link_offset<6, 1>(L.vp, 1 - p, 0, fwd_h(L, h, S, mu)), gn);
    gram_schmidt(gn);
    v2<T>* q = U + link_offset<NC>(L.vp, p, mu, h);
    load_link_f64<T, NC>(q, A);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Cx<double> f = cmul(g.e[a][0], A.e[0][b]);
        f = cmac(f, g.e[a][1], A.e[1][b]);
        B.e[a][b] = cmac(f, g.e[a][2], A.e[2][b]);
      }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Cx<double> f = cx<double>(0, 0);
        f = cmac_cb(f, B.e[a][0], gn.e[b][0]);
        f = cmac_cb(f, B.e[a][1], gn.e[b][1]);
        A.e[a][b] = cmac_cb(f, B.e[a][2], gn.e[b][2]);
      }
    store_link_from_f64<T, NC>(q, A);
  }
}

// bandwidth probes: 16-byte elements, one per thread
static __global__ __launch_bounds__(kBlock) void k_probe_copy(const double2* __restrict__ a,
                                                       double2* __restrict__ b, const size_t n) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = a[i];
}
static __global__ __launch_bounds__(kBlock) void k_probe_rmw(v2<double>* __restrict__ b, const size_t n) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  v2<double> v = __builtin_nontemporal_load(b + i);
  v.x *= 2.0;
  v.y *= 2.0;
  __builtin_nontemporal_store(v, b + i);
}
static __global__ __launch_bounds__(kBlock) void k_probe_read(const double2* __restrict__ a,
                                                       double* __restrict__ out, const size_t n) {
  __shared__ double lds[kBlock / 64];
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double acc = 0;
  if (i < n) acc = a[i].x + a[i].y;
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

static __global__ __launch_bounds__(kBlock) void k_philox(const uint32_t* __restrict__ ctr,
                                                   uint32_t* __restrict__ out, const int64_t n,
                                                   const uint32_t k0, const uint32_t k1) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const U4 r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[4 * i + k] = r.v[k];
}

}  // namespace gf
