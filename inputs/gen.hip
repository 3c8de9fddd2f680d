// gen.hip -- seeded synthetic SU(3) gauge fields for tests and benchmarks.
//
// This module produces INPUTS only. It holds none of the gauge-fixing
// arithmetic (no overrelaxation, functional, precision, annealing or
// reunitarisation code); the GPU library and the CPU oracle both take its
// fields as given. Every random number comes from Philox4x32-10 (Salmon,
// Moraes, Dror, Shaw, SC'11), keyed by (seed low, seed high) with counter
// (index, stream, tag, attempt), so the host and the device entry points
// produce the same field from the same seed.
//
// Field layout (canonical): complex128 U[s][mu][3][3],
// s = ((t*nz + z)*ny + y)*nx + x, dims = {nt, nz, ny, nx}, mu = 0:t 1:x 2:y 3:z.
//
// Recipes:
//  * smooth field: V_mu(x) = exp(i eps H), H traceless Hermitian whose
//    independent real components are N(0,1) (Box-Muller) before the trace
//    is removed; then a Haar-random gauge transformation h(x):
//    U_mu(x) = h(x) V_mu(x) h(x+mu)^dagger.
//  * Haar SU(3): two rows of complex N(0,1) entries, Gram-Schmidt, third row
//    conj(row0 x row1); the law is invariant under right multiplication by
//    SU(3), hence Haar.
//  * pure gauge: U_mu(x) = h(x) h(x+mu)^dagger.
//  * quenched Wilson-action heatbath (Creutz / Cabibbo-Marinari with the
//    Kennedy-Pendleton SU(2) sampler, Phys. Lett. B 156 (1985) 393), cold
//    start, phases mu = 0..3 x parity 0, 1 per sweep; action
//    S = beta sum_P (1 - Re tr U_P / 3).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#define GEN_HD __host__ __device__ inline

namespace gen {

struct cx {
  double re, im;
};
struct m3 {
  cx e[3][3];
};

GEN_HD cx mk(double r, double i) {
  cx z;
  z.re = r;
  z.im = i;
  return z;
}
GEN_HD cx add(cx a, cx b) { return mk(a.re + b.re, a.im + b.im); }
GEN_HD cx sub(cx a, cx b) { return mk(a.re - b.re, a.im - b.im); }
GEN_HD cx mul(cx a, cx b) { return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
GEN_HD cx cj(cx a) { return mk(a.re, -a.im); }
GEN_HD cx scl(cx a, double s) { return mk(a.re * s, a.im * s); }

GEN_HD m3 zero3() {
  m3 A;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) A.e[a][b] = mk(0.0, 0.0);
  return A;
}
GEN_HD m3 unit3() {
  m3 A = zero3();
  for (int a = 0; a < 3; ++a) A.e[a][a] = mk(1.0, 0.0);
  return A;
}
GEN_HD m3 mm(const m3& A, const m3& B) {
  m3 C;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cx acc = mk(0.0, 0.0);
      for (int k = 0; k < 3; ++k) acc = add(acc, mul(A.e[a][k], B.e[k][b]));
      C.e[a][b] = acc;
    }
  return C;
}
GEN_HD m3 dag(const m3& A) {
  m3 C;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C.e[a][b] = cj(A.e[b][a]);
  return C;
}
GEN_HD m3 madd(const m3& A, const m3& B) {
  m3 C;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C.e[a][b] = add(A.e[a][b], B.e[a][b]);
  return C;
}

GEN_HD m3 load(const double* U, int64_t link) {
  m3 A;
  const double* p = U + link * 18;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) A.e[a][b] = mk(p[(3 * a + b) * 2], p[(3 * a + b) * 2 + 1]);
  return A;
}
GEN_HD void store(double* U, int64_t link, const m3& A) {
  double* p = U + link * 18;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      p[(3 * a + b) * 2] = A.e[a][b].re;
      p[(3 * a + b) * 2 + 1] = A.e[a][b].im;
    }
}

// ---- Philox4x32-10 --------------------------------------------------------
GEN_HD void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                   uint32_t out[4]) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}
GEN_HD double u01(uint32_t u) { return ((double)u + 0.5) * (1.0 / 4294967296.0); }

GEN_HD void uniforms(uint64_t seed, uint32_t idx, uint32_t stream, uint32_t tag, uint32_t attempt,
                     double u[4]) {
  uint32_t r[4];
  philox(idx, stream, tag, attempt, (uint32_t)seed, (uint32_t)(seed >> 32), r);
  for (int k = 0; k < 4; ++k) u[k] = u01(r[k]);
}

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Box-Muller: 4 uniforms -> 4 standard normals
GEN_HD void gaussians(uint64_t seed, uint32_t idx, uint32_t stream, uint32_t tag, double g[4]) {
  double u[4];
  uniforms(seed, idx, stream, tag, 0u, u);
  const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
  g[0] = r0 * cos(kTwoPi * u[1]);
  g[1] = r0 * sin(kTwoPi * u[1]);
  g[2] = r1 * cos(kTwoPi * u[3]);
  g[3] = r1 * sin(kTwoPi * u[3]);
}

enum : uint32_t {
  kTagHeatbath = 0x2000u,  // | mu << 8 | kind << 4 | subgroup
  kTagSmooth = 0x3000u,    // | block
  kTagHaar = 0x4000u,      // | block
};

// Haar-random SU(3) for (site, copy)
GEN_HD m3 haar_su3(uint64_t seed, uint32_t site, uint32_t copy) {
  double g[12];
  for (int blk = 0; blk < 3; ++blk) gaussians(seed, site, copy, kTagHaar | (uint32_t)blk, g + 4 * blk);
  m3 A = zero3();
  for (int b = 0; b < 3; ++b) {
    A.e[0][b] = mk(g[2 * b], g[2 * b + 1]);
    A.e[1][b] = mk(g[6 + 2 * b], g[6 + 2 * b + 1]);
  }
  double n0 = 0.0;
  for (int b = 0; b < 3; ++b) n0 += A.e[0][b].re * A.e[0][b].re + A.e[0][b].im * A.e[0][b].im;
  n0 = 1.0 / sqrt(n0);
  for (int b = 0; b < 3; ++b) A.e[0][b] = scl(A.e[0][b], n0);
  cx ip = mk(0.0, 0.0);
  for (int b = 0; b < 3; ++b) ip = add(ip, mul(cj(A.e[0][b]), A.e[1][b]));
  for (int b = 0; b < 3; ++b) A.e[1][b] = sub(A.e[1][b], mul(ip, A.e[0][b]));
  double n1 = 0.0;
  for (int b = 0; b < 3; ++b) n1 += A.e[1][b].re * A.e[1][b].re + A.e[1][b].im * A.e[1][b].im;
  n1 = 1.0 / sqrt(n1);
  for (int b = 0; b < 3; ++b) A.e[1][b] = scl(A.e[1][b], n1);
  A.e[2][0] = cj(sub(mul(A.e[0][1], A.e[1][2]), mul(A.e[0][2], A.e[1][1])));
  A.e[2][1] = cj(sub(mul(A.e[0][2], A.e[1][0]), mul(A.e[0][0], A.e[1][2])));
  A.e[2][2] = cj(sub(mul(A.e[0][0], A.e[1][1]), mul(A.e[0][1], A.e[1][0])));
  return A;
}

// exp(A) by Taylor series with scaling and squaring (A = i eps H, |A| ~ 1)
GEN_HD m3 expm(const m3& A0) {
  double nrm = 0.0;
  for (int a = 0; a < 3; ++a) {
    double row = 0.0;
    for (int b = 0; b < 3; ++b) row += fabs(A0.e[a][b].re) + fabs(A0.e[a][b].im);
    nrm = row > nrm ? row : nrm;
  }
  int k = 0;
  while (nrm > 0.25 && k < 30) {
    nrm *= 0.5;
    ++k;
  }
  m3 A = A0;
  const double sc = ldexp(1.0, -k);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) A.e[a][b] = scl(A.e[a][b], sc);
  m3 E = unit3(), term = unit3();
  for (int n = 1; n <= 20; ++n) {
    term = mm(term, A);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) term.e[a][b] = scl(term.e[a][b], 1.0 / (double)n);
    E = madd(E, term);
  }
  for (int i = 0; i < k; ++i) E = mm(E, E);
  return E;
}

// V = exp(i eps H) for link (site, mu)
GEN_HD m3 smooth_link(uint64_t seed, uint32_t site, int mu, double eps) {
  double g[12];
  for (int blk = 0; blk < 3; ++blk)
    gaussians(seed, site, (uint32_t)mu, kTagSmooth | (uint32_t)blk, g + 4 * blk);
  // H: diagonal g0..g2, off-diagonal (0,1),(0,2),(1,2) = g3+i g4, g5+i g6, g7+i g8
  m3 H = zero3();
  H.e[0][0] = mk(g[0], 0.0);
  H.e[1][1] = mk(g[1], 0.0);
  H.e[2][2] = mk(g[2], 0.0);
  H.e[0][1] = mk(g[3], g[4]);
  H.e[1][0] = mk(g[3], -g[4]);
  H.e[0][2] = mk(g[5], g[6]);
  H.e[2][0] = mk(g[5], -g[6]);
  H.e[1][2] = mk(g[7], g[8]);
  H.e[2][1] = mk(g[7], -g[8]);
  const double tr3 = (g[0] + g[1] + g[2]) / 3.0;
  for (int a = 0; a < 3; ++a) H.e[a][a].re -= tr3;
  m3 A;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) A.e[a][b] = mk(-eps * H.e[a][b].im, eps * H.e[a][b].re);  // i eps H
  return expm(A);
}

// ---- geometry ---------------------------------------------------------------
struct Lat {
  int64_t ext[4];  // by direction: t, x, y, z
  int64_t V;
};
inline Lat make_lat(const int32_t dims[4]) {
  Lat L;
  L.ext[0] = dims[0];
  L.ext[1] = dims[3];
  L.ext[2] = dims[2];
  L.ext[3] = dims[1];
  L.V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
  return L;
}
GEN_HD void coords(const Lat& L, int64_t s, int64_t c[4]) {
  c[1] = s % L.ext[1];
  s /= L.ext[1];
  c[2] = s % L.ext[2];
  s /= L.ext[2];
  c[3] = s % L.ext[3];
  s /= L.ext[3];
  c[0] = s;
}
GEN_HD int64_t index(const Lat& L, const int64_t c[4]) {
  return ((c[0] * L.ext[3] + c[3]) * L.ext[2] + c[2]) * L.ext[1] + c[1];
}
GEN_HD int64_t shift(const Lat& L, int64_t s, int mu, int step) {
  int64_t c[4];
  coords(L, s, c);
  c[mu] = (c[mu] + step + L.ext[mu]) % L.ext[mu];
  return index(L, c);
}
GEN_HD int parity(const Lat& L, int64_t s) {
  int64_t c[4];
  coords(L, s, c);
  return (int)((c[0] + c[1] + c[2] + c[3]) & 1);
}

// ---- Wilson heatbath link update ------------------------------------------------
GEN_HD m3 embed(const double a[4], int i, int j) {
  m3 G = unit3();
  G.e[i][i] = mk(a[0], a[3]);
  G.e[i][j] = mk(a[2], a[1]);
  G.e[j][i] = mk(-a[2], a[1]);
  G.e[j][j] = mk(a[0], -a[3]);
  return G;
}

GEN_HD void heatbath_link(double* U, const Lat& L, int64_t s, int mu, double beta, uint64_t seed,
                          uint32_t sweep) {
  m3 A = zero3();  // staple sum
  const int64_t sp = shift(L, s, mu, +1);
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    const int64_t sn = shift(L, s, nu, +1), sm = shift(L, s, nu, -1);
    const int64_t spm = shift(L, sp, nu, -1);
    m3 up = mm(mm(load(U, sp * 4 + nu), dag(load(U, sn * 4 + mu))), dag(load(U, s * 4 + nu)));
    m3 dn = mm(mm(dag(load(U, spm * 4 + nu)), dag(load(U, sm * 4 + mu))), load(U, sm * 4 + nu));
    A = madd(A, madd(up, dn));
  }
  m3 Ul = load(U, s * 4 + mu);
  m3 W = mm(Ul, A);
  const int SI[3] = {0, 0, 1}, SJ[3] = {1, 2, 2};
  for (int sg = 0; sg < 3; ++sg) {
    const int i = SI[sg], j = SJ[sg];
    // quaternion part of the (i,j) block of W^dag: maximiser direction of Re tr[g W]
    const cx wii = cj(W.e[i][i]), wij = cj(W.e[j][i]), wji = cj(W.e[i][j]), wjj = cj(W.e[j][j]);
    double q[4] = {0.5 * (wii.re + wjj.re), 0.5 * (wij.im + wji.im), 0.5 * (wij.re - wji.re),
                   0.5 * (wii.im - wjj.im)};
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (n < 1e-150) continue;
    const double alpha = (beta / 3.0) * 2.0 * n;
    const uint32_t tagkp = kTagHeatbath | ((uint32_t)mu << 8) | (0u << 4) | (uint32_t)sg;
    const uint32_t tagdir = kTagHeatbath | ((uint32_t)mu << 8) | (1u << 4) | (uint32_t)sg;
    double lam2 = -1.0;
    for (uint32_t att = 0; att < 1024u; ++att) {
      double u[4];
      uniforms(seed, (uint32_t)s, sweep, tagkp, att, u);
      const double c = cos(kTwoPi * u[1]);
      const double l2 = -(log(u[0]) + c * c * log(u[2])) / (2.0 * alpha);
      if (u[3] * u[3] <= 1.0 - l2) {
        lam2 = l2;
        break;
      }
    }
    if (lam2 < 0.0) continue;  // attempt cap hit: leave the link unchanged in this subgroup
    double d[4];
    uniforms(seed, (uint32_t)s, sweep, tagdir, 0u, d);
    const double cth = 2.0 * d[0] - 1.0;
    const double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
    const double phi = kTwoPi * d[1];
    const double rad = 2.0 * sqrt(lam2 * (1.0 - lam2));  // sqrt(1 - X0^2) without cancellation
    const double X[4] = {1.0 - 2.0 * lam2, rad * sth * cos(phi), rad * sth * sin(phi), rad * cth};
    const double qh[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
    const m3 G = mm(embed(X, i, j), embed(qh, i, j));
    Ul = mm(G, Ul);
    W = mm(G, W);
  }
  store(U, s * 4 + mu, Ul);
}

GEN_HD m3 config0_link(uint64_t seed, const Lat& L, int64_t s, int mu, double eps) {
  const m3 V = smooth_link(seed, (uint32_t)s, mu, eps);
  const m3 h = haar_su3(seed, (uint32_t)s, 0u);
  const m3 hn = haar_su3(seed, (uint32_t)shift(L, s, mu, +1), 0u);
  return mm(mm(h, V), dag(hn));
}

// ---- device kernels -----------------------------------------------------------
__global__ void k_unit(double* U, int64_t nlinks) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlinks) return;
  store(U, l, unit3());
}

__global__ void k_config0(double* U, Lat L, double eps, uint64_t seed) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= 4 * L.V) return;
  const int64_t s = l >> 2;
  const int mu = (int)(l & 3);
  store(U, l, config0_link(seed, L, s, mu, eps));
}

// U_mu(x) <- h(x) U_mu(x) h(x+mu)^dag with Haar h from (seed, copy); each thread
// owns the four forward links of one site, so the update is in place and race-free.
__global__ void k_haar_copy(double* U, Lat L, uint64_t seed, uint32_t copy) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= L.V) return;
  const m3 h = haar_su3(seed, (uint32_t)s, copy);
  for (int mu = 0; mu < 4; ++mu) {
    const m3 hn = haar_su3(seed, (uint32_t)shift(L, s, mu, +1), copy);
    store(U, s * 4 + mu, mm(mm(h, load(U, s * 4 + mu)), dag(hn)));
  }
}

// config-0 links written straight into the gauge-fixing library's device
// layout (its public header documents it), for lattices whose canonical FP64
// form would not fit in device memory: complex element (p, mu, c, h) at
//   p*4*nc*vp + (h/W)*W*4*nc + (mu*nc + c)*W + h%W,   W = kLayoutTile,
// p = parity of the site, h = s >> 1, c = 3a + b < nc (nc = 6: rows 0 and 1;
// nc = 9: all rows), vp = V/2 rounded up to a multiple of W; T = float or
// double, re and im interleaved. The link values are those of k_config0,
// rounded to T.
constexpr int64_t kLayoutTile = 2048;  // sites per tile of the documented layout

template <typename T>
__device__ void config0_packed_link(T* F, const Lat& L, int nc, int64_t vp, double eps,
                                    uint64_t seed, int64_t l) {
  const int64_t s = l >> 2;
  const int mu = (int)(l & 3);
  const m3 A = config0_link(seed, L, s, mu, eps);
  int64_t c4[4];
  coords(L, s, c4);
  const int64_t p = (c4[0] + c4[1] + c4[2] + c4[3]) & 1;
  const int64_t h = s >> 1;
  const int64_t W = kLayoutTile;
  const int64_t base = p * 4 * nc * vp + (h / W) * W * 4 * nc + (int64_t)mu * nc * W + h % W;
  for (int c = 0; c < nc; ++c) {
    T* q = F + 2 * (base + (int64_t)c * W);
    q[0] = (T)A.e[c / 3][c % 3].re;
    q[1] = (T)A.e[c / 3][c % 3].im;
  }
}

// Grid-stride over the 4V links: a launch holds fewer than 2^32 work-items.
template <typename T>
__global__ void k_config0_packed(T* F, Lat L, int nc, int64_t vp, double eps, uint64_t seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < 4 * L.V; l += stride)
    config0_packed_link(F, L, nc, vp, eps, seed, l);
}

// one heatbath phase: links U_mu(x) with x of the given parity (their staples
// only involve links that this phase does not change)
__global__ void k_heatbath(double* U, Lat L, int mu, int par, double beta, uint64_t seed,
                           uint32_t sweep) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= L.V / 2) return;
  // half index h -> the site of parity `par` among the pair (2h, 2h+1)
  int64_t s = 2 * h;
  if (parity(L, s) != par) s += 1;
  heatbath_link(U, L, s, mu, beta, seed, sweep);
}

}  // namespace gen

using namespace gen;

static int dims_ok(const int32_t* dims) {
  if (!dims) return 0;
  for (int k = 0; k < 4; ++k)
    if (dims[k] < 2 || (dims[k] & 1)) return 0;
  return 1;
}

extern "C" {

// ---- host entry points (host memory) -----------------------------------------
int gen_unit_field(double* U, const int32_t dims[4]) {
  if (!U || !dims_ok(dims)) return -1;
  const Lat L = make_lat(dims);
  for (int64_t l = 0; l < 4 * L.V; ++l) store(U, l, unit3());
  return 0;
}

int gen_haar_sites(double* g, const int32_t dims[4], uint64_t seed, uint32_t copy) {
  if (!g || !dims_ok(dims)) return -1;
  const Lat L = make_lat(dims);
  for (int64_t s = 0; s < L.V; ++s) store(g, s, haar_su3(seed, (uint32_t)s, copy));
  return 0;
}

int gen_smooth_links(double* U, const int32_t dims[4], double eps, uint64_t seed) {
  if (!U || !dims_ok(dims)) return -1;
  const Lat L = make_lat(dims);
  for (int64_t s = 0; s < L.V; ++s)
    for (int mu = 0; mu < 4; ++mu) store(U, s * 4 + mu, smooth_link(seed, (uint32_t)s, mu, eps));
  return 0;
}

int gen_config0(double* U, const int32_t dims[4], double eps, uint64_t seed) {
  if (!U || !dims_ok(dims)) return -1;
  const Lat L = make_lat(dims);
  for (int64_t s = 0; s < L.V; ++s)
    for (int mu = 0; mu < 4; ++mu) store(U, s * 4 + mu, config0_link(seed, L, s, mu, eps));
  return 0;
}

int gen_pure_gauge(double* U, const int32_t dims[4], uint64_t seed) {
  if (!U || !dims_ok(dims)) return -1;
  const Lat L = make_lat(dims);
  for (int64_t s = 0; s < L.V; ++s) {
    const m3 h = haar_su3(seed, (uint32_t)s, 0u);
    for (int mu = 0; mu < 4; ++mu)
      store(U, s * 4 + mu, mm(h, dag(haar_su3(seed, (uint32_t)shift(L, s, mu, +1), 0u))));
  }
  return 0;
}

int gen_haar_copy(double* U, const int32_t dims[4], uint64_t seed, uint32_t copy) {
  if (!U || !dims_ok(dims)) return -1;
  const Lat L = make_lat(dims);
  for (int64_t s = 0; s < L.V; ++s) {
    const m3 h = haar_su3(seed, (uint32_t)s, copy);
    for (int mu = 0; mu < 4; ++mu) {
      const m3 hn = haar_su3(seed, (uint32_t)shift(L, s, mu, +1), copy);
      store(U, s * 4 + mu, mm(mm(h, load(U, s * 4 + mu)), dag(hn)));
    }
  }
  return 0;
}

int gen_heatbath_sweep(double* U, const int32_t dims[4], double beta, uint64_t seed,
                       uint32_t sweep) {
  if (!U || !dims_ok(dims) || !(beta > 0.0)) return -1;
  const Lat L = make_lat(dims);
  for (int mu = 0; mu < 4; ++mu)
    for (int par = 0; par < 2; ++par)
      for (int64_t s = 0; s < L.V; ++s)
        if (parity(L, s) == par) heatbath_link(U, L, s, mu, beta, seed, sweep);
  return 0;
}

void gen_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1], out);
}

// ---- device entry points (device memory, enqueued on `stream`) ---------------------
static int launch_status() { return hipGetLastError() == hipSuccess ? 0 : -4; }
// clears a stale per-thread error left by an earlier, unrelated runtime call
static void clear_stale_error() { (void)hipGetLastError(); }

int gen_gpu_unit_field(double* U, const int32_t dims[4], void* stream) {
  if (!U || !dims_ok(dims)) return -1;
  const Lat L = make_lat(dims);
  const int64_t n = 4 * L.V;
  clear_stale_error();
  hipLaunchKernelGGL(k_unit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     U, n);
  return launch_status();
}

int gen_gpu_config0(double* U, const int32_t dims[4], double eps, uint64_t seed, void* stream) {
  if (!U || !dims_ok(dims)) return -1;
  const Lat L = make_lat(dims);
  const int64_t n = 4 * L.V;
  clear_stale_error();
  hipLaunchKernelGGL(k_config0, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, U, L, eps, seed);
  return launch_status();
}

// prec_bytes 4 (float) or 8 (double); nc 6 or 9; F holds 8 * vp * 2*nc * prec_bytes bytes
int gen_gpu_config0_packed(void* F, const int32_t dims[4], int32_t prec_bytes, int32_t nc,
                           double eps, uint64_t seed, void* stream) {
  if (!F || !dims_ok(dims) || (prec_bytes != 4 && prec_bytes != 8) || (nc != 6 && nc != 9))
    return -1;
  const Lat L = make_lat(dims);
  if (L.V > ((int64_t)1 << 30)) return -1;
  const int64_t vp = (L.V / 2 + kLayoutTile - 1) / kLayoutTile * kLayoutTile;
  const int64_t n = 4 * L.V;
  const int64_t want = (n + 255) / 256;
  const unsigned blocks = (unsigned)(want < (1 << 20) ? want : (1 << 20));
  clear_stale_error();
  if (prec_bytes == 4)
    hipLaunchKernelGGL(k_config0_packed<float>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (float*)F, L, (int)nc, vp, eps, seed);
  else
    hipLaunchKernelGGL(k_config0_packed<double>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (double*)F, L, (int)nc, vp, eps, seed);
  return launch_status();
}

int gen_gpu_haar_copy(double* U, const int32_t dims[4], uint64_t seed, uint32_t copy,
                      void* stream) {
  if (!U || !dims_ok(dims)) return -1;
  const Lat L = make_lat(dims);
  clear_stale_error();
  hipLaunchKernelGGL(k_haar_copy, dim3((unsigned)((L.V + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, U, L, seed, copy);
  return launch_status();
}

int gen_gpu_heatbath_sweep(double* U, const int32_t dims[4], double beta, uint64_t seed,
                           uint32_t sweep, void* stream) {
  if (!U || !dims_ok(dims) || !(beta > 0.0)) return -1;
  const Lat L = make_lat(dims);
  const int64_t nh = L.V / 2;
  clear_stale_error();
  for (int mu = 0; mu < 4; ++mu)
    for (int par = 0; par < 2; ++par)
      hipLaunchKernelGGL(k_heatbath, dim3((unsigned)((nh + 127) / 128)), dim3(128), 0,
                         (hipStream_t)stream, U, L, mu, par, beta, seed, sweep);
  return launch_status();
}

}  // extern "C"
