/*
 * oracle.c -- plain FP64 CPU oracle for checkerboard overrelaxation gauge
 * fixing and simulated annealing (Schroeck & Vogt, arXiv:1209.4008).
 *
 * TEST INFRASTRUCTURE. This file is the independent reference that the GPU
 * library is checked against. It is called only from the test suite, the
 * smoke check and the CPU baseline leg of the benchmark. It shares no code
 * (no headers, helpers, tables or constants) with the GPU library.
 *
 * Style: plain loops over full 3x3 complex matrices, written from the
 * defining equations: a site's update gathers the eight links that g(x)
 * moves (eq. (4)), maximises the local functional Re tr[g(x) K(x)] (K of
 * eq. (5)) within each SU(2) subgroup of SU(3) in turn (eq. (6)), with the
 * update rule of the method (overrelaxation, heatbath, microcanonical), and
 * writes the links back. There is no blocking, fusion or reordering, so that
 * a reader can check each step against the paper by eye. Compiled -O2
 * -ffp-contract=off (no FMA contraction, no fast-math); OpenMP only splits
 * the sites of one checkerboard sublattice, which share no link, and all
 * reductions are summed serially in site order (results do not depend on
 * the thread count).
 *
 * Passages followed (sections/equations of the paper):
 *   eq. (4)  gauge transformation U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dagger
 *   eq. (3)  Landau gauge functional F_g = Re sum_{mu,x} tr U^g_mu(x)
 *   eq. (5)  K(x) = sum_mu U_mu(x) g(x+mu)^dag + U_mu(x-mu)^dag g(x-mu)^dag
 *   eq. (6)  SU(2) local solution g = K^dag / sqrt(det K^dag), applied in the
 *            three SU(2) subgroups of SU(3) (Sec. 2, Cabibbo-Marinari)
 *   Sec. 2   overrelaxation g -> g^omega, omega in [1, 2)
 *   Sec. 2   RED/BLACK checkerboard decomposition
 *   eq. (7)  precision theta = (1/(V N_c)) sum_x tr[Delta(x) Delta(x)^dag]
 *   Alg. 1   the iteration: sweep one sublattice, then the other, until
 *            theta is below the target
 *   Sec. 1   simulated annealing as a preconditioner; Coulomb gauge
 * Points where the paper is silent are filled with the readings documented
 * next to the code that uses them (degenerate subgroups, theta's Delta,
 * normalisation of F, form of g^omega, annealing weight and sampler).
 */
#include "or.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* complex numbers and 3x3 complex matrices                                   */
/* ------------------------------------------------------------------------- */
typedef struct { double re, im; } cx;
typedef struct { cx m[3][3]; } mat3;

static cx cx_make(double re, double im) { cx z; z.re = re; z.im = im; return z; }
static cx cx_add(cx a, cx b) { return cx_make(a.re + b.re, a.im + b.im); }
static cx cx_sub(cx a, cx b) { return cx_make(a.re - b.re, a.im - b.im); }
static cx cx_mul(cx a, cx b) { return cx_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static cx cx_conj(cx a) { return cx_make(a.re, -a.im); }
static double cx_abs2(cx a) { return a.re * a.re + a.im * a.im; }

static mat3 mat_zero(void) { mat3 A; memset(&A, 0, sizeof A); return A; }
static mat3 mat_unit(void) {
  mat3 A = mat_zero();
  for (int a = 0; a < 3; ++a) A.m[a][a] = cx_make(1.0, 0.0);
  return A;
}
static mat3 mat_mul(const mat3* A, const mat3* B) {
  mat3 C;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cx acc = cx_make(0.0, 0.0);
      for (int k = 0; k < 3; ++k) acc = cx_add(acc, cx_mul(A->m[a][k], B->m[k][b]));
      C.m[a][b] = acc;
    }
  return C;
}
static mat3 mat_dag(const mat3* A) {
  mat3 C;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C.m[a][b] = cx_conj(A->m[b][a]);
  return C;
}
static mat3 mat_add(const mat3* A, const mat3* B) {
  mat3 C;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C.m[a][b] = cx_add(A->m[a][b], B->m[a][b]);
  return C;
}
static double mat_retr(const mat3* A) { return A->m[0][0].re + A->m[1][1].re + A->m[2][2].re; }

/* ------------------------------------------------------------------------- */
/* geometry: periodic 4D lattice, s = ((t*nz + z)*ny + y)*nx + x              */
/* ------------------------------------------------------------------------- */
typedef struct {
  int64_t ext[4]; /* extent along direction mu: t, x, y, z */
  int64_t V;
} lat_t;

int or_check_dims(const int32_t dims[4]) {
  if (!dims) return -1;
  for (int k = 0; k < 4; ++k)
    if (dims[k] < 2 || (dims[k] & 1)) return -1; /* checkerboard needs even extents */
  return 0;
}

int64_t or_volume(const int32_t dims[4]) {
  return (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
}

static lat_t make_lat(const int32_t dims[4]) {
  lat_t L;
  L.ext[0] = dims[0]; /* t */
  L.ext[1] = dims[3]; /* x */
  L.ext[2] = dims[2]; /* y */
  L.ext[3] = dims[1]; /* z */
  L.V = or_volume(dims);
  return L;
}

static void site_coords(const lat_t* L, int64_t s, int64_t c[4]) {
  c[1] = s % L->ext[1]; s /= L->ext[1];
  c[2] = s % L->ext[2]; s /= L->ext[2];
  c[3] = s % L->ext[3]; s /= L->ext[3];
  c[0] = s;
}

static int64_t site_index(const lat_t* L, const int64_t c[4]) {
  return ((c[0] * L->ext[3] + c[3]) * L->ext[2] + c[2]) * L->ext[1] + c[1];
}

static int site_parity(const lat_t* L, int64_t s) {
  int64_t c[4];
  site_coords(L, s, c);
  return (int)((c[0] + c[1] + c[2] + c[3]) & 1);
}

/* neighbour x + step*mu_hat with periodic wrap */
static int64_t neighbour(const lat_t* L, int64_t s, int mu, int step) {
  int64_t c[4];
  site_coords(L, s, c);
  c[mu] = (c[mu] + step + L->ext[mu]) % L->ext[mu];
  return site_index(L, c);
}

/* ------------------------------------------------------------------------- */
/* link access in the canonical layout U[s][mu][3][3]                         */
/* ------------------------------------------------------------------------- */
static mat3 get_link(const double* U, int64_t s, int mu) {
  mat3 A;
  const double* p = U + ((s * 4 + mu) * 9) * 2;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) A.m[a][b] = cx_make(p[(3 * a + b) * 2], p[(3 * a + b) * 2 + 1]);
  return A;
}

static void put_link(double* U, int64_t s, int mu, const mat3* A) {
  double* p = U + ((s * 4 + mu) * 9) * 2;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      p[(3 * a + b) * 2] = A->m[a][b].re;
      p[(3 * a + b) * 2 + 1] = A->m[a][b].im;
    }
}

static mat3 mat_from18(const double M[18]) {
  mat3 A;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) A.m[a][b] = cx_make(M[(3 * a + b) * 2], M[(3 * a + b) * 2 + 1]);
  return A;
}

static void mat_to18(const mat3* A, double M[18]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      M[(3 * a + b) * 2] = A->m[a][b].re;
      M[(3 * a + b) * 2 + 1] = A->m[a][b].im;
    }
}

/* ------------------------------------------------------------------------- */
/* SU(2) subgroups of SU(3) (Sec. 2, Cabibbo-Marinari)                        */
/* ------------------------------------------------------------------------- */
/* Subgroup order (0,1), (0,2), (1,2): the paper does not fix it. */
static const int SG_I[3] = {0, 0, 1};
static const int SG_J[3] = {1, 2, 2};

/* Quaternion part of the (i,j) block, for the convention
 *   a <-> [[a0 + i a3, a2 + i a1], [-a2 + i a1, a0 - i a3]].
 * Any 2x2 complex block B splits as B = Q(a) + i Q(b) with real quaternions
 * a, b; only a contributes to Re tr[g B] for g in SU(2), and a is what is
 * returned here. For B in R * SU(2) the block equals Q(a). */
void or_su2_part(const double M18[18], int i, int j, double q[4]) {
  mat3 M = mat_from18(M18);
  cx bii = M.m[i][i], bij = M.m[i][j], bji = M.m[j][i], bjj = M.m[j][j];
  q[0] = 0.5 * (bii.re + bjj.re);
  q[1] = 0.5 * (bij.im + bji.im);
  q[2] = 0.5 * (bij.re - bji.re);
  q[3] = 0.5 * (bii.im - bjj.im);
}

/* Embed the SU(2) element with quaternion a into SU(3) at rows/cols (i,j). */
static mat3 embed_su2(const double a[4], int i, int j) {
  mat3 G = mat_unit();
  G.m[i][i] = cx_make(a[0], a[3]);
  G.m[i][j] = cx_make(a[2], a[1]);
  G.m[j][i] = cx_make(-a[2], a[1]);
  G.m[j][j] = cx_make(a[0], -a[3]);
  return G;
}

/* Below this |q|^2 the subgroup is skipped (G = 1): the paper does not say
 * what to do with a vanishing local sum. */
#define OR_DEGENERATE 1e-300

/* Overrelaxation (Sec. 2): replace the local maximum g = q/|q| by g^omega.
 * The paper leaves the form of the power open beyond saying that it is a
 * low-order expansion; the reading used here is the one whose operation
 * count equals the paper's count for this step (Alg. 1). It works on the
 * unnormalised q = (q0, qv):
 *   b = (omega q0^2 + |qv|^2) / (q0^2 + |qv|^2),
 *   c = 1 / sqrt(q0^2 + b^2 |qv|^2),
 *   s = (c q0, b c qv),
 * which is unit-norm, equals q/|q| exactly at omega = 1, and for
 * q ~ (cos phi, sin phi n) rotates by phi' with
 * tan phi' = (1 + (omega-1) cos^2 phi) tan phi, i.e. phi' = omega phi to
 * first order in phi. */
int or_overrelax(const double q[4], double omega, double s[4]) {
  double a0sq = q[0] * q[0];
  double avsq = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  if (a0sq + avsq < OR_DEGENERATE) return -1;
  double b = (omega * a0sq + avsq) / (a0sq + avsq);
  double c = 1.0 / sqrt(a0sq + b * b * avsq);
  s[0] = c * q[0];
  s[1] = b * c * q[1];
  s[2] = b * c * q[2];
  s[3] = b * c * q[3];
  return 0;
}

/* Other forms of the power g^omega of the local maximum g = q/|q| (Sec. 2:
 * the exponentiation is carried out to first or second order). Writing
 * g = 1 + a, the binomial series (1 + a)^omega is truncated:
 *   form 1: 1 + omega a,
 *   form 2: 1 + omega a + omega (omega - 1)/2 a^2,
 * and the result is projected back onto SU(2), i.e. the quaternion is divided
 * by its length. In quaternion components, with a = (g0 - 1, gv) and
 * a^2 = (a0^2 - |gv|^2, 2 a0 gv), form 2 is
 *   (1 + omega a0 + omega (omega - 1)/2 (a0^2 - |gv|^2), gv (omega + omega (omega - 1) a0)).
 *   form 3: the exact power: g = (cos phi, n sin phi) -> (cos(omega phi),
 *   n sin(omega phi)), phi = atan2(|gv|, g0) in [0, pi]; for gv = 0 the power
 *   is left at g (phi = 0 or pi, no axis).
 * form 0 is or_overrelax. Returns -1 if |q| (or the truncated series) is
 * degenerate. */
int or_overrelax_form(const double q[4], double omega, int form, double s[4]) {
  if (form == 0) return or_overrelax(q, omega, s);
  if (form < 0 || form > 3) return -1;
  double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  if (n2 < OR_DEGENERATE) return -1;
  double n = sqrt(n2);
  double g[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
  double gv2 = g[1] * g[1] + g[2] * g[2] + g[3] * g[3];
  double t[4];
  if (form == 3) {
    double nv = sqrt(gv2);
    if (nv == 0.0) {
      for (int k = 0; k < 4; ++k) s[k] = g[k];
      return 0;
    }
    double phi = atan2(nv, g[0]);
    double f = sin(omega * phi) / nv;
    t[0] = cos(omega * phi);
    t[1] = f * g[1];
    t[2] = f * g[2];
    t[3] = f * g[3];
  } else {
    double a0 = g[0] - 1.0;
    double c2 = form == 2 ? 0.5 * omega * (omega - 1.0) : 0.0;
    t[0] = 1.0 + omega * a0 + c2 * (a0 * a0 - gv2);
    double fv = omega + 2.0 * c2 * a0;
    t[1] = fv * g[1];
    t[2] = fv * g[2];
    t[3] = fv * g[3];
  }
  double m2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2] + t[3] * t[3];
  if (m2 < OR_DEGENERATE) return -1;
  double m = sqrt(m2);
  for (int k = 0; k < 4; ++k) s[k] = t[k] / m;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as     */
/* easy as 1, 2, 3", SC'11): 10 rounds of the Philox S-box on a 4x32 counter  */
/* with a 2x32 key bumped by the Weyl constants between rounds.               */
/* ------------------------------------------------------------------------- */
void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in (0, 1): (u + 1/2) 2^-32 */
static double u01(uint32_t u) { return ((double)u + 0.5) * (1.0 / 4294967296.0); }

/* Counter layout of the annealing draws (one Philox block per use):
 *   key = (seed low 32 bits, seed high 32 bits)
 *   ctr = (site index, sweep low 32 bits, tag, attempt)
 *   tag = 0x1000 | kind << 8 | subgroup; kind 0 = KP trial, 1 = direction. */
#define OR_TAG_KP(sg) (0x1000u | (0u << 8) | (uint32_t)(sg))
#define OR_TAG_DIR(sg) (0x1000u | (1u << 8) | (uint32_t)(sg))
#define OR_TAG_SR(sg) (0x1000u | (2u << 8) | (uint32_t)(sg))
#define OR_KP_MAX_ATTEMPTS 1024

static void draw_block(uint64_t seed, uint64_t site, uint64_t sweep, uint32_t tag,
                       uint32_t attempt, double u[4]) {
  uint32_t ctr[4] = {(uint32_t)site, (uint32_t)sweep, tag, attempt};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t r[4];
  or_philox4x32(ctr, key, r);
  for (int k = 0; k < 4; ++k) u[k] = u01(r[k]);
}

/* Accept decisions of the heatbath, seen from outside. A sampler working in
 * lower precision takes the same decisions as this one except where the
 * margin m = (1 - lambda^2) - u4^2 of a trial is within its rounding of 0.
 * With a control block, every trial whose |m| is below tau is recorded (in
 * the order the trials are made: subgroup, then attempt), the trials listed
 * in flip are decided the other way, and the smallest |m| met is kept. */
#define OR_HB_MAX_FLIPS 8
#define OR_HB_MAX_SEEN 16
typedef struct {
  double tau;
  int nflip;
  int flip_sg[OR_HB_MAX_FLIPS], flip_att[OR_HB_MAX_FLIPS];
  int nseen;
  int seen_sg[OR_HB_MAX_SEEN], seen_att[OR_HB_MAX_SEEN];
  double min_margin;
} hb_ctl;

static int hb_flipped(const hb_ctl* c, int sg, int att) {
  for (int k = 0; k < c->nflip; ++k)
    if (c->flip_sg[k] == sg && c->flip_att[k] == att) return 1;
  return 0;
}

/* Kennedy & Pendleton, Phys. Lett. B 156 (1985) 393: with
 * lambda^2 = -(ln u1 + cos^2(2 pi u2) ln u3) / (2 alpha) (a Gamma(3/2)
 * variate scaled by 1/(2 alpha)), accept when u4^2 <= 1 - lambda^2 and set
 * X0 = 1 - 2 lambda^2; X0 then has density ~ sqrt(1 - X0^2) exp(alpha X0).
 * Returns the attempts used (0 when the cap was hit) and lambda^2. */
static int kp_lambda2(double alpha, uint64_t seed, uint64_t site, uint64_t sweep, int sg,
                      hb_ctl* ctl, double* lam2_out) {
  const double two_pi = 6.283185307179586476925286766559;
  for (int a = 0; a < OR_KP_MAX_ATTEMPTS; ++a) {
    double u[4];
    draw_block(seed, site, sweep, OR_TAG_KP(sg), (uint32_t)a, u);
    double cs = cos(two_pi * u[1]);
    double lam2 = -(log(u[0]) + cs * cs * log(u[2])) / (2.0 * alpha);
    int accept = u[3] * u[3] <= 1.0 - lam2;
    if (ctl) {
      double m = fabs((1.0 - lam2) - u[3] * u[3]);
      if (m < ctl->min_margin) ctl->min_margin = m;
      if (m < ctl->tau && ctl->nseen < OR_HB_MAX_SEEN) {
        ctl->seen_sg[ctl->nseen] = sg;
        ctl->seen_att[ctl->nseen] = a;
        ctl->nseen++;
      }
      if (hb_flipped(ctl, sg, a)) accept = !accept;
    }
    if (accept) {
      /* a trial accepted against its margin may sit just above 1 */
      *lam2_out = lam2 > 1.0 ? 1.0 : lam2;
      return a + 1;
    }
  }
  return 0;
}

int or_kp_draw(double alpha, uint64_t seed, uint64_t site, uint64_t sweep, int sg, double* X0) {
  double lam2;
  int n = kp_lambda2(alpha, seed, site, sweep, sg, NULL, &lam2);
  if (n) *X0 = 1.0 - 2.0 * lam2;
  return n;
}

/* SU(2) element X with density ~ exp(alpha X0) under Haar measure: X0 from
 * the Kennedy-Pendleton draw, (X1, X2, X3) uniform on the sphere of radius
 * sqrt(1 - X0^2) from one more Philox block (cos theta = 2 u1 - 1,
 * phi = 2 pi u2). Returns the attempts used, 0 if the cap was hit. */
static int heatbath_su2(double alpha, uint64_t seed, uint64_t site, uint64_t sweep, int sg,
                        hb_ctl* ctl, double X[4]) {
  double lam2;
  int n = kp_lambda2(alpha, seed, site, sweep, sg, ctl, &lam2);
  if (n == 0) return 0;
  const double two_pi = 6.283185307179586476925286766559;
  double d[4];
  draw_block(seed, site, sweep, OR_TAG_DIR(sg), 0u, d);
  double cth = 2.0 * d[0] - 1.0;
  double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
  double phi = two_pi * d[1];
  /* sqrt(1 - X0^2) = 2 lambda sqrt(1 - lambda^2) for X0 = 1 - 2 lambda^2,
   * written without the cancellation of 1 - X0^2 near X0 = 1 */
  double rad = 2.0 * sqrt(lam2 * (1.0 - lam2));
  X[0] = 1.0 - 2.0 * lam2;
  X[1] = rad * sth * cos(phi);
  X[2] = rad * sth * sin(phi);
  X[3] = rad * cth;
  return n;
}

int or_heatbath_su2(double alpha, uint64_t seed, uint64_t site, uint64_t sweep, int sg,
                    double X[4]) {
  return heatbath_su2(alpha, seed, site, sweep, sg, NULL, X);
}

/* ------------------------------------------------------------------------- */
/* the local problem at one site                                              */
/* ------------------------------------------------------------------------- */
/* By eq. (4) a transformation g(x) at the single site x moves exactly eight
 * links: U_mu(x) -> g(x) U_mu(x) and U_mu(x - mu) -> U_mu(x - mu) g(x)^dag,
 * mu = 0..3. Only these enter the part of F (eq. (3)) that depends on g(x),
 * so a site's update reads them, works on them and writes them back. */
typedef struct {
  mat3 fwd[4]; /* U_mu(x)      */
  mat3 bwd[4]; /* U_mu(x - mu) */
} site_links;

static void gather_site(const double* U, const lat_t* L, int64_t s, site_links* S) {
  for (int mu = 0; mu < 4; ++mu) {
    S->fwd[mu] = get_link(U, s, mu);
    S->bwd[mu] = get_link(U, neighbour(L, s, mu, -1), mu);
  }
}

static void scatter_site(double* U, const lat_t* L, int64_t s, const site_links* S) {
  for (int mu = 0; mu < 4; ++mu) {
    put_link(U, s, mu, &S->fwd[mu]);
    put_link(U, neighbour(L, s, mu, -1), mu, &S->bwd[mu]);
  }
}

/* First direction entering K, F and theta: Landau all four, Coulomb the
 * spatial ones (Sec. 1: Coulomb gauge d_i A_i = 0). */
static int first_dir(int gauge) { return gauge == OR_COULOMB ? 1 : 0; }

/* K(x) of eq. (5) from the current links: sum over mu in D of
 * U_mu(x) + U_mu(x - mu)^dag. Every update is applied to the field in place,
 * so the transformations g(x +- mu) that eq. (5) writes out are already in
 * the neighbouring links. With it the g(x)-dependent part of F is
 * Re tr[g(x) K(x)]. */
static mat3 site_K(const site_links* S, int gauge) {
  mat3 K = mat_zero();
  for (int mu = first_dir(gauge); mu < 4; ++mu) {
    mat3 Wd = mat_dag(&S->bwd[mu]);
    K = mat_add(&K, &S->fwd[mu]);
    K = mat_add(&K, &Wd);
  }
  return K;
}

static mat3 local_K(const double* U, const lat_t* L, int gauge, int64_t s) {
  site_links S;
  gather_site(U, L, s, &S);
  return site_K(&S, gauge);
}

void or_local_K(const double* U, const int32_t dims[4], int gauge, int64_t s, double K[18]) {
  lat_t L = make_lat(dims);
  mat3 Km = local_K(U, &L, gauge, s);
  mat_to18(&Km, K);
}

/* eq. (4) at x for a factor h of g(x): g(x) -> h g(x). All four directions
 * move, also in the Coulomb gauge (the output stays a gauge transform of the
 * input). */
static void transform_site(site_links* S, const mat3* h) {
  mat3 hd = mat_dag(h);
  for (int mu = 0; mu < 4; ++mu) {
    S->fwd[mu] = mat_mul(h, &S->fwd[mu]);
    S->bwd[mu] = mat_mul(&S->bwd[mu], &hd);
  }
}

/* ------------------------------------------------------------------------- */
/* site updates: overrelaxation, heatbath, microcanonical, stochastic        */
/* ------------------------------------------------------------------------- */
enum { UPD_OR = 0, UPD_HB = 1, UPD_MICRO = 2, UPD_SR = 3 };
typedef struct {
  int kind;
  double omega;
  double T;     /* heatbath temperature; stochastic relaxation: probability p */
  uint64_t seed, sweep;
  int form;     /* overrelaxation: form of g^omega (0: or_overrelax) */
} upd_t;

/* The element of subgroup sg = (i,j) by which the update rule moves g(x),
 * given the current K. For h = embed(a) in the subgroup,
 * Re tr[h K] = 2 a.q + (terms without a), q the quaternion part of the (i,j)
 * block of K^dag (or_su2_part); by eq. (6) its maximum over SU(2) is at
 * a = q/|q|. Returns 0 with h set, 1 when the heatbath hit its attempt cap,
 * -1 when the subgroup is degenerate (h = 1 in both cases). */
static int subgroup_element(const mat3* K, int sg, int64_t s, const upd_t* u, hb_ctl* ctl,
                            mat3* h) {
  const int i = SG_I[sg], j = SG_J[sg];
  mat3 Kd = mat_dag(K);
  double M18[18], q[4], g[4];
  mat_to18(&Kd, M18);
  or_su2_part(M18, i, j, q);
  double qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  if (qn2 < OR_DEGENERATE) return -1;
  int kind = u->kind;
  if (kind == UPD_SR) {
    /* stochastic relaxation (Sec. 1): with probability p the
     * microcanonical step, otherwise the (over)relaxation step */
    double d[4];
    draw_block(u->seed, (uint64_t)s, u->sweep, OR_TAG_SR(sg), 0u, d);
    kind = d[0] < u->T ? UPD_MICRO : UPD_OR;
  }
  if (kind == UPD_OR) {
    /* the local maximum raised to omega (Sec. 2, overrelaxation) */
    if (or_overrelax_form(q, u->omega, u->form, g) < 0) return -1;
    *h = embed_su2(g, i, j);
    return 0;
  }
  double n = sqrt(qn2);
  double qh[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
  mat3 Gh = embed_su2(qh, i, j);
  if (kind == UPD_MICRO) {
    /* the reflection through the local maximum, ghat^2: Re tr[h K] is
     * unchanged */
    *h = mat_mul(&Gh, &Gh);
    return 0;
  }
  /* heatbath with weight exp(Re tr[h K] / T): writing h = X qhat,
   * Re tr[h K] = 2|q| X0 + const, so X is drawn with density ~ exp(alpha X0)
   * under Haar measure, alpha = 2|q|/T */
  double X[4];
  if (heatbath_su2(2.0 * n / u->T, u->seed, (uint64_t)s, u->sweep, sg, ctl, X) == 0) return 1;
  mat3 GX = embed_su2(X, i, j);
  *h = mat_mul(&GX, &Gh);
  return 0;
}

/* One site's update: g(x) is moved within the SU(2) subgroups of SU(3) one
 * after another (Cabibbo-Marinari; subgroup order (0,1), (0,2), (1,2)), each
 * step taking K of eq. (5) from the links as the previous steps left them.
 * gtot (may be NULL) receives the product of the three factors, i.e. the
 * whole change of g(x). Returns the number of heatbath steps that hit the
 * attempt cap. */
static int update_site(site_links* S, int gauge, int64_t s, const upd_t* u, hb_ctl* ctl,
                       mat3* gtot) {
  int capped = 0;
  if (gtot) *gtot = mat_unit();
  for (int sg = 0; sg < 3; ++sg) {
    mat3 K = site_K(S, gauge);
    mat3 h;
    int rc = subgroup_element(&K, sg, s, u, ctl, &h);
    if (rc != 0) {
      capped += rc > 0;
      continue;
    }
    transform_site(S, &h);
    if (gtot) *gtot = mat_mul(&h, gtot);
  }
  return capped;
}

static int site_update(double* U, const lat_t* L, int gauge, int64_t s, const upd_t* u,
                       mat3* gtot) {
  site_links S;
  gather_site(U, L, s, &S);
  int capped = update_site(&S, gauge, s, u, NULL, gtot);
  scatter_site(U, L, s, &S);
  return capped;
}

/* g may be NULL; else g[s] receives the site's total transformation (sites of
 * the other parity: 1) */
static int half_sweep(double* U, const int32_t dims[4], int gauge, int parity, const upd_t* u,
                      int64_t* n_capped, double* g) {
  if (!U || or_check_dims(dims) != 0 || (parity != 0 && parity != 1)) return -1;
  if (gauge != OR_LANDAU && gauge != OR_COULOMB) return -1;
  lat_t L = make_lat(dims);
  int64_t capped = 0;
  /* Sec. 2: all sites of one sublattice are independent (no shared link) */
#pragma omp parallel for schedule(static) reduction(+ : capped)
  for (int64_t s = 0; s < L.V; ++s) {
    mat3 gs = mat_unit();
    if (site_parity(&L, s) == parity) capped += site_update(U, &L, gauge, s, u, &gs);
    if (g) mat_to18(&gs, g + 18 * s);
  }
  if (n_capped) *n_capped += capped;
  return 0;
}

/* Overrelaxation update of the listed sites only, each as in a half-sweep
 * (all listed sites must have the same parity, so that none shares a link).
 * Used to check large lattices on a sample of sites. */
int or_update_sites(double* U, const int32_t dims[4], int gauge, double omega,
                    const int64_t* sites, int64_t n) {
  if (!U || !sites || or_check_dims(dims) != 0 || !(omega >= 1.0 && omega < 2.0)) return -1;
  lat_t L = make_lat(dims);
  if (n <= 0) return 0;
  int p0 = site_parity(&L, sites[0]);
  for (int64_t k = 0; k < n; ++k)
    if (sites[k] < 0 || sites[k] >= L.V || site_parity(&L, sites[k]) != p0) return -1;
  upd_t u = {UPD_OR, omega, 0.0, 0, 0, 0};
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) site_update(U, &L, gauge, sites[k], &u, NULL);
  return 0;
}

/* Heatbath update (annealing step at temperature T, draws keyed by seed and
 * sweep) of the listed sites of one parity only (sampled checks). */
int or_heatbath_sites(double* U, const int32_t dims[4], int gauge, double T, uint64_t seed,
                      uint64_t sweep, const int64_t* sites, int64_t n) {
  if (!U || !sites || or_check_dims(dims) != 0 || !(T > 0.0)) return -1;
  lat_t L = make_lat(dims);
  if (n <= 0) return 0;
  int p0 = site_parity(&L, sites[0]);
  for (int64_t k = 0; k < n; ++k)
    if (sites[k] < 0 || sites[k] >= L.V || site_parity(&L, sites[k]) != p0) return -1;
  upd_t u = {UPD_HB, 0.0, T, seed, sweep, 0};
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) site_update(U, &L, gauge, sites[k], &u, NULL);
  return 0;
}

/* Every result the heatbath update of site s can have when each trial whose
 * accept margin is below tau may be decided either way (see hb_ctl). The
 * outcomes are explored depth first: outcome 0 is the exact one; every other
 * takes one more borderline trial the other way than an outcome before it,
 * a trial met after the last one flipped there. Each outcome is the site's 8
 * links, U_mu(s) for mu = 0..3 then U_mu(s - mu), 18 doubles each. Returns the
 * number of outcomes (at most max_out; the field is not changed), or -1. */
int or_heatbath_site_outcomes(const double* U, const int32_t dims[4], int gauge, double T,
                              uint64_t seed, uint64_t sweep, int64_t s, double tau, int max_out,
                              double* links_out, double* min_margin) {
  if (!U || !links_out || or_check_dims(dims) != 0 || !(T > 0.0) || max_out < 1) return -1;
  if (gauge != OR_LANDAU && gauge != OR_COULOMB) return -1;
  lat_t L = make_lat(dims);
  if (s < 0 || s >= L.V) return -1;
  upd_t u = {UPD_HB, 0.0, T, seed, sweep, 0};
  site_links S0;
  gather_site(U, &L, s, &S0);
  /* pending flip sets, processed in order */
  enum { QMAX = 256 };
  int qn[QMAX], qsg[QMAX][OR_HB_MAX_FLIPS], qatt[QMAX][OR_HB_MAX_FLIPS];
  int head = 0, tail = 1, nout = 0;
  qn[0] = 0;
  while (head < tail && nout < max_out) {
    hb_ctl c;
    memset(&c, 0, sizeof c);
    c.tau = tau;
    c.min_margin = HUGE_VAL;
    c.nflip = qn[head];
    for (int k = 0; k < c.nflip; ++k) {
      c.flip_sg[k] = qsg[head][k];
      c.flip_att[k] = qatt[head][k];
    }
    site_links S = S0;
    update_site(&S, gauge, s, &u, &c, NULL);
    double* o = links_out + (size_t)nout * 8 * 18;
    for (int mu = 0; mu < 4; ++mu) {
      mat_to18(&S.fwd[mu], o + 18 * mu);
      mat_to18(&S.bwd[mu], o + 18 * (4 + mu));
    }
    if (nout == 0 && min_margin) *min_margin = c.min_margin;
    ++nout;
    /* children: flip one more borderline trial met after the last flip */
    int lsg = c.nflip ? c.flip_sg[c.nflip - 1] : -1;
    int latt = c.nflip ? c.flip_att[c.nflip - 1] : -1;
    for (int k = 0; k < c.nseen; ++k) {
      int sg = c.seen_sg[k], att = c.seen_att[k];
      if (sg < lsg || (sg == lsg && att <= latt)) continue;
      if (c.nflip >= OR_HB_MAX_FLIPS || tail >= QMAX) break;
      qn[tail] = c.nflip + 1;
      for (int m = 0; m < c.nflip; ++m) {
        qsg[tail][m] = c.flip_sg[m];
        qatt[tail][m] = c.flip_att[m];
      }
      qsg[tail][c.nflip] = sg;
      qatt[tail][c.nflip] = att;
      ++tail;
    }
    ++head;
  }
  return nout;
}

int or_sweep(double* U, const int32_t dims[4], int gauge, int parity, double omega) {
  if (!(omega >= 1.0 && omega < 2.0)) return -1; /* Sec. 2: omega in [1, 2) */
  upd_t u = {UPD_OR, omega, 0.0, 0, 0, 0};
  return half_sweep(U, dims, gauge, parity, &u, NULL, NULL);
}

int or_sweep_form(double* U, const int32_t dims[4], int gauge, int parity, double omega,
                  int form) {
  if (!(omega >= 1.0 && omega < 2.0) || form < 0 || form > 3) return -1;
  upd_t u = {UPD_OR, omega, 0.0, 0, 0, form};
  return half_sweep(U, dims, gauge, parity, &u, NULL, NULL);
}

int or_sweep_sr(double* U, const int32_t dims[4], int gauge, int parity, double omega,
                double prob, uint64_t seed, uint64_t sweep) {
  if (!(omega >= 1.0 && omega < 2.0) || !(prob >= 0.0 && prob <= 1.0)) return -1;
  upd_t u = {UPD_SR, omega, prob, seed, sweep, 0};
  return half_sweep(U, dims, gauge, parity, &u, NULL, NULL);
}

int or_micro_half(double* U, const int32_t dims[4], int gauge, int parity) {
  upd_t u = {UPD_MICRO, 0.0, 0.0, 0, 0, 0};
  return half_sweep(U, dims, gauge, parity, &u, NULL, NULL);
}

int or_heatbath_half(double* U, const int32_t dims[4], int gauge, int parity, double T,
                     uint64_t seed, uint64_t sweep, int64_t* n_capped) {
  if (!(T > 0.0) || !isfinite(T)) return -1;
  upd_t u = {UPD_HB, 0.0, T, seed, sweep, 0};
  return half_sweep(U, dims, gauge, parity, &u, n_capped, NULL);
}

int or_half_sweep_g(double* U, const int32_t dims[4], int gauge, int parity, int kind,
                    double omega, double param, uint64_t seed, uint64_t sweep, double* g) {
  upd_t u = {kind, omega, param, seed, sweep, 0};
  if (!g) return -1;
  if (kind == UPD_OR || kind == UPD_SR) {
    if (!(omega >= 1.0 && omega < 2.0)) return -1;
    if (kind == UPD_SR && !(param >= 0.0 && param <= 1.0)) return -1;
  } else if (kind == UPD_HB) {
    if (!(param > 0.0) || !isfinite(param)) return -1;
  } else if (kind != UPD_MICRO) {
    return -1;
  }
  return half_sweep(U, dims, gauge, parity, &u, NULL, g);
}

int or_anneal_sweep(double* U, const int32_t dims[4], int gauge, double T, uint64_t seed,
                    uint64_t sweep, int n_micro, int64_t* n_capped) {
  if (n_micro < 0) return -1;
  int rc = 0;
  for (int p = 0; p < 2 && rc == 0; ++p)
    rc = or_heatbath_half(U, dims, gauge, p, T, seed, sweep, n_capped);
  for (int k = 0; k < n_micro && rc == 0; ++k)
    for (int p = 0; p < 2 && rc == 0; ++p) rc = or_micro_half(U, dims, gauge, p);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* reductions                                                                 */
/* ------------------------------------------------------------------------- */
double or_functional_raw(const double* U, const int32_t dims[4], int gauge) {
  lat_t L = make_lat(dims);
  double* per_site = (double*)malloc(sizeof(double) * (size_t)L.V);
  int mu0 = first_dir(gauge);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < L.V; ++s) {
    double acc = 0.0;
    for (int mu = mu0; mu < 4; ++mu) {
      mat3 A = get_link(U, s, mu);
      acc += mat_retr(&A);
    }
    per_site[s] = acc;
  }
  double sum = 0.0;
  for (int64_t s = 0; s < L.V; ++s) sum += per_site[s];
  free(per_site);
  return sum;
}

/* Eq. (3), normalised by N_c |D| V (Landau) or N_c |D| V_s per timeslice
 * (Coulomb) so that the unit field gives exactly 1; the paper prints the
 * unnormalised sum. */
double or_functional(const double* U, const int32_t dims[4], int gauge, double* out) {
  lat_t L = make_lat(dims);
  int mu0 = first_dir(gauge);
  double* per_site = (double*)malloc(sizeof(double) * (size_t)L.V);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < L.V; ++s) {
    double acc = 0.0;
    for (int mu = mu0; mu < 4; ++mu) {
      mat3 A = get_link(U, s, mu);
      acc += mat_retr(&A);
    }
    per_site[s] = acc;
  }
  double ret;
  if (gauge == OR_LANDAU) {
    double sum = 0.0;
    for (int64_t s = 0; s < L.V; ++s) sum += per_site[s];
    ret = sum / (3.0 * 4.0 * (double)L.V);
    if (out) out[0] = ret;
  } else {
    int64_t nt = L.ext[0], Vs = L.V / nt;
    double mean = 0.0;
    for (int64_t t = 0; t < nt; ++t) {
      double sum = 0.0;
      for (int64_t k = 0; k < Vs; ++k) sum += per_site[t * Vs + k];
      double Ft = sum / (3.0 * 3.0 * (double)Vs);
      if (out) out[t] = Ft;
      mean += Ft;
    }
    ret = mean / (double)nt;
  }
  free(per_site);
  return ret;
}

/* Hermitian traceless part of (M - M^dag)/(2i): for M = U_mu(x) this is the
 * lattice gauge potential A_mu(x) (U = exp(i a g A), eq. (2), to first order). */
static mat3 traceless_antiherm(const mat3* M) {
  mat3 A;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cx d = cx_sub(M->m[a][b], cx_conj(M->m[b][a])); /* M - M^dag */
      A.m[a][b] = cx_make(0.5 * d.im, -0.5 * d.re);   /* divided by 2i */
    }
  double tr3 = (A.m[0][0].re + A.m[1][1].re + A.m[2][2].re) / 3.0;
  for (int a = 0; a < 3; ++a) A.m[a][a].re -= tr3;
  return A;
}

static double tr_MMdag(const mat3* M) {
  double acc = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) acc += cx_abs2(M->m[a][b]);
  return acc;
}

/* Sum per-site contributions to theta (eq. (7)): Landau (1/(N_c V)) sum_x,
 * Coulomb per timeslice (1/(N_c V_s)) sum_{x in t}. */
static double finish_theta(const lat_t* L, int gauge, const double* per_site, double* out) {
  if (gauge == OR_LANDAU) {
    double sum = 0.0;
    for (int64_t s = 0; s < L->V; ++s) sum += per_site[s];
    double th = sum / (3.0 * (double)L->V);
    if (out) out[0] = th;
    return th;
  }
  int64_t nt = L->ext[0], Vs = L->V / nt;
  double mx = 0.0;
  for (int64_t t = 0; t < nt; ++t) {
    double sum = 0.0;
    for (int64_t k = 0; k < Vs; ++k) sum += per_site[t * Vs + k];
    double th = sum / (3.0 * (double)Vs);
    if (out) out[t] = th;
    if (th > mx) mx = th;
  }
  return mx;
}

/* The paper uses Delta^g without defining it. Reading: the lattice
 * divergence Delta(x) = sum_{mu in D} [A_mu(x) - A_mu(x - mu)] of the gauge
 * potential of the current (already transformed) links. */
double or_theta_A(const double* U, const int32_t dims[4], int gauge, double* out) {
  lat_t L = make_lat(dims);
  int mu0 = first_dir(gauge);
  double* per_site = (double*)malloc(sizeof(double) * (size_t)L.V);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < L.V; ++s) {
    mat3 D = mat_zero();
    for (int mu = mu0; mu < 4; ++mu) {
      mat3 Uf = get_link(U, s, mu);
      mat3 Ub = get_link(U, neighbour(&L, s, mu, -1), mu);
      mat3 Af = traceless_antiherm(&Uf);
      mat3 Ab = traceless_antiherm(&Ub);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          D.m[a][b] = cx_add(D.m[a][b], cx_sub(Af.m[a][b], Ab.m[a][b]));
    }
    per_site[s] = tr_MMdag(&D);
  }
  double ret = finish_theta(&L, gauge, per_site, out);
  free(per_site);
  return ret;
}

/* Same quantity from K(x) of eq. (5): (K - K^dag)/(2i) equals
 * sum_mu [(U_mu(x) - U_mu(x)^dag) - (U_mu(x-mu) - U_mu(x-mu)^dag)]/(2i),
 * so its traceless part is Delta(x). */
double or_theta_K(const double* U, const int32_t dims[4], int gauge, double* out) {
  lat_t L = make_lat(dims);
  double* per_site = (double*)malloc(sizeof(double) * (size_t)L.V);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < L.V; ++s) {
    mat3 K = local_K(U, &L, gauge, s);
    mat3 D = traceless_antiherm(&K);
    per_site[s] = tr_MMdag(&D);
  }
  double ret = finish_theta(&L, gauge, per_site, out);
  free(per_site);
  return ret;
}

/* Gram-Schmidt projection onto SU(3): normalise row 0, orthogonalise and
 * normalise row 1, row 2 = conj(row0 x row1). The paper does not state how
 * links are kept unitary; the last formula is also how a link stored as its
 * first two rows is completed (Sec. 4.1, 12-real storage). */
void or_reunitarize(double* U, int64_t n_links) {
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < n_links; ++l) {
    double* p = U + l * 18;
    mat3 A = mat_from18(p);
    double n0 = 0.0;
    for (int b = 0; b < 3; ++b) n0 += cx_abs2(A.m[0][b]);
    n0 = 1.0 / sqrt(n0);
    for (int b = 0; b < 3; ++b) A.m[0][b] = cx_make(A.m[0][b].re * n0, A.m[0][b].im * n0);
    cx ip = cx_make(0.0, 0.0); /* <row0, row1> = sum conj(u0) u1 */
    for (int b = 0; b < 3; ++b) ip = cx_add(ip, cx_mul(cx_conj(A.m[0][b]), A.m[1][b]));
    for (int b = 0; b < 3; ++b) A.m[1][b] = cx_sub(A.m[1][b], cx_mul(ip, A.m[0][b]));
    double n1 = 0.0;
    for (int b = 0; b < 3; ++b) n1 += cx_abs2(A.m[1][b]);
    n1 = 1.0 / sqrt(n1);
    for (int b = 0; b < 3; ++b) A.m[1][b] = cx_make(A.m[1][b].re * n1, A.m[1][b].im * n1);
    A.m[2][0] = cx_conj(cx_sub(cx_mul(A.m[0][1], A.m[1][2]), cx_mul(A.m[0][2], A.m[1][1])));
    A.m[2][1] = cx_conj(cx_sub(cx_mul(A.m[0][2], A.m[1][0]), cx_mul(A.m[0][0], A.m[1][2])));
    A.m[2][2] = cx_conj(cx_sub(cx_mul(A.m[0][0], A.m[1][1]), cx_mul(A.m[0][1], A.m[1][0])));
    mat_to18(&A, p);
  }
}

/* Unitarity deviation: the largest modulus of an element of U U^dag - 1 over
 * all links (the definition, with full 3x3 products); NaN gives +Inf. */
double or_unitarity(const double* U, const int32_t dims[4]) {
  lat_t L = make_lat(dims);
  double worst = 0.0;
  for (int64_t s = 0; s < L.V; ++s)
    for (int mu = 0; mu < 4; ++mu) {
      mat3 A = get_link(U, s, mu);
      mat3 Ad = mat_dag(&A);
      mat3 P = mat_mul(&A, &Ad);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double re = P.m[a][b].re - (a == b ? 1.0 : 0.0), im = P.m[a][b].im;
          double m = sqrt(re * re + im * im);
          if (m != m) return HUGE_VAL;
          if (m > worst) worst = m;
        }
    }
  return worst;
}

double or_plaquette(const double* U, const int32_t dims[4]) {
  lat_t L = make_lat(dims);
  double* per_site = (double*)malloc(sizeof(double) * (size_t)L.V);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < L.V; ++s) {
    double acc = 0.0;
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        mat3 A = get_link(U, s, mu);
        mat3 B = get_link(U, neighbour(&L, s, mu, +1), nu);
        mat3 C = get_link(U, neighbour(&L, s, nu, +1), mu);
        mat3 D = get_link(U, s, nu);
        mat3 Cd = mat_dag(&C), Dd = mat_dag(&D);
        mat3 AB = mat_mul(&A, &B);
        mat3 ABC = mat_mul(&AB, &Cd);
        mat3 P = mat_mul(&ABC, &Dd);
        acc += mat_retr(&P) / 3.0;
      }
    per_site[s] = acc;
  }
  double sum = 0.0;
  for (int64_t s = 0; s < L.V; ++s) sum += per_site[s];
  free(per_site);
  return sum / (6.0 * (double)L.V);
}

/* eq. (4): U_mu(x) <- g(x) U_mu(x) g(x + mu)^dagger */
int or_gauge_transform(double* U, const int32_t dims[4], const double* g) {
  if (!U || !g || or_check_dims(dims) != 0) return -1;
  lat_t L = make_lat(dims);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < L.V; ++s) {
    mat3 gx = mat_from18(g + s * 18);
    for (int mu = 0; mu < 4; ++mu) {
      mat3 gn = mat_from18(g + neighbour(&L, s, mu, +1) * 18);
      mat3 gnd = mat_dag(&gn);
      mat3 A = get_link(U, s, mu);
      mat3 B = mat_mul(&gx, &A);
      mat3 C = mat_mul(&B, &gnd);
      put_link(U, s, mu, &C);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* driver: the while-theta loop of Alg. 1 with a check every check_every      */
/* sweeps (Sec. 4.1 checks F_g and theta after every 100th iteration)        */
/* ------------------------------------------------------------------------- */
int or_fix(double* U, const int32_t dims[4], int gauge, double omega, int form,
           double theta_target, int32_t max_sweeps, int32_t check_every,
           int32_t reunit_at_check, int32_t* sweeps_out, double* F_out, double* theta_out) {
  if (!U || or_check_dims(dims) != 0 || check_every < 1 || max_sweeps < 0) return -1;
  if (!(omega >= 1.0 && omega < 2.0) || form < 0 || form > 3) return -1;
  int64_t V = or_volume(dims);
  int32_t sweeps = 0;
  int converged = 0;
  double F = 0.0, th = 0.0;
  for (;;) {
    if (sweeps > 0 && reunit_at_check) or_reunitarize(U, V * 4);
    F = or_functional(U, dims, gauge, NULL);
    th = or_theta_K(U, dims, gauge, NULL);
    if (th < theta_target) { converged = 1; break; }
    if (sweeps >= max_sweeps) break;
    for (int32_t k = 0; k < check_every && sweeps < max_sweeps; ++k) {
      or_sweep_form(U, dims, gauge, 0, omega, form);
      or_sweep_form(U, dims, gauge, 1, omega, form);
      ++sweeps;
    }
  }
  if (sweeps_out) *sweeps_out = sweeps;
  if (F_out) *F_out = F;
  if (theta_out) *theta_out = th;
  return converged ? 0 : 1;
}

/* Coulomb gauge (Sec. 1: the condition on the spatial components only) with
 * converged timeslices frozen, a driver the paper does not describe: the
 * timeslices are independent gauge-fixing problems (K, F and theta of a timeslice involve its
 * spatial links only), so at every check each timeslice whose theta_t is
 * below the target stops being swept; its spatial links then stay as they
 * are, while the temporal links it shares with a timeslice still being swept
 * keep receiving that timeslice's transformations. Stops when every theta_t
 * is below the target (all frozen) or at max_sweeps. F_out and theta_out
 * receive nt values each; frozen_at (may be NULL) receives, per timeslice,
 * the sweep count at which it was frozen (-1 if never). */
int or_fix_coulomb_frozen(double* U, const int32_t dims[4], double omega, double theta_target,
                          int32_t max_sweeps, int32_t check_every, int32_t reunit_at_check,
                          int32_t* sweeps_out, double* F_out, double* theta_out,
                          int32_t* frozen_at) {
  if (!U || or_check_dims(dims) != 0 || check_every < 1 || max_sweeps < 0) return -1;
  if (!(omega >= 1.0 && omega < 2.0) || !F_out || !theta_out) return -1;
  lat_t L = make_lat(dims);
  const int64_t nt = L.ext[0], Vs = L.V / nt;
  unsigned char* active = (unsigned char*)malloc((size_t)nt);
  for (int64_t t = 0; t < nt; ++t) {
    active[t] = 1;
    if (frozen_at) frozen_at[t] = -1;
  }
  int32_t sweeps = 0;
  int converged = 0;
  upd_t u = {UPD_OR, omega, 0.0, 0, 0, 0};
  for (;;) {
    if (sweeps > 0 && reunit_at_check) or_reunitarize(U, L.V * 4);
    or_functional(U, dims, OR_COULOMB, F_out);
    or_theta_K(U, dims, OR_COULOMB, theta_out);
    int n_active = 0;
    for (int64_t t = 0; t < nt; ++t) {
      if (active[t] && theta_out[t] < theta_target) {
        active[t] = 0;
        if (frozen_at) frozen_at[t] = sweeps;
      }
      n_active += active[t];
    }
    if (n_active == 0) { converged = 1; break; }
    if (sweeps >= max_sweeps) break;
    for (int32_t k = 0; k < check_every && sweeps < max_sweeps; ++k) {
      for (int parity = 0; parity < 2; ++parity) {
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < L.V; ++s)
          if (site_parity(&L, s) == parity && active[s / Vs])
            site_update(U, &L, OR_COULOMB, s, &u, NULL);
      }
      ++sweeps;
    }
  }
  free(active);
  if (sweeps_out) *sweeps_out = sweeps;
  return converged ? 0 : 1;
}

/* ------------------------------------------------------------------------- */
/* maximally Abelian gauge (named in Sec. 1 and the summary; the paper does   */
/* not write out its functional): maximise                                    */
/*   R[U] = sum_{x, mu} sum_k |U_mu(x)_kk|^2,                                 */
/* the weight of the diagonal (Abelian) part of the links.                    */
/* ------------------------------------------------------------------------- */

/* R of the 8 links at site s after the local transformation G = embed(a) on
 * the subgroup (i, j): U_mu(s) -> G U_mu(s), U_mu(s - mu) -> U_mu(s - mu) G^dag.
 * a need not be a unit quaternion (embed is linear in a on the (i, j) block). */
static double mag_local_R(const double* U, const lat_t* L, int64_t s, const double a[4], int i,
                          int j) {
  mat3 G = embed_su2(a, i, j);
  mat3 Gd = mat_dag(&G);
  double R = 0.0;
  for (int mu = 0; mu < 4; ++mu) {
    mat3 Uf = get_link(U, s, mu);
    mat3 Ub = get_link(U, neighbour(L, s, mu, -1), mu);
    mat3 A = mat_mul(&G, &Uf);
    mat3 B = mat_mul(&Ub, &Gd);
    for (int k = 0; k < 3; ++k) R += cx_abs2(A.m[k][k]) + cx_abs2(B.m[k][k]);
  }
  return R;
}

/* R is a quadratic form in a plus a constant (the diagonal entries outside
 * the subgroup do not depend on a): R(a) = a^T M a + C with C = R(0). M by
 * polarisation: M_kk = R(e_k) - C, M_kl = (R(e_k + e_l) - R(e_k) - R(e_l) + C)/2. */
static void mag_matrix(const double* U, const lat_t* L, int64_t s, int sg, double M[4][4]) {
  int i = SG_I[sg], j = SG_J[sg];
  double zero[4] = {0, 0, 0, 0};
  double C = mag_local_R(U, L, s, zero, i, j);
  double Rk[4];
  for (int k = 0; k < 4; ++k) {
    double e[4] = {0, 0, 0, 0};
    e[k] = 1.0;
    Rk[k] = mag_local_R(U, L, s, e, i, j);
    M[k][k] = Rk[k] - C;
  }
  for (int k = 0; k < 4; ++k)
    for (int l = k + 1; l < 4; ++l) {
      double e[4] = {0, 0, 0, 0};
      e[k] = 1.0;
      e[l] = 1.0;
      M[k][l] = M[l][k] = 0.5 * (mag_local_R(U, L, s, e, i, j) - Rk[k] - Rk[l] + C);
    }
}

void or_mag_matrix(const double* U, const int32_t dims[4], int64_t s, int sg, double M[16]) {
  lat_t L = make_lat(dims);
  double A[4][4];
  mag_matrix(U, &L, s, sg, A);
  for (int k = 0; k < 4; ++k)
    for (int l = 0; l < 4; ++l) M[4 * k + l] = A[k][l];
}

/* Eigenvector of the largest eigenvalue of a real symmetric 3x3 matrix by
 * cyclic Jacobi rotations (Golub & Van Loan, Matrix Computations, Sec. 8.5):
 * each rotation zeroes one off-diagonal entry; sweeps repeat until the
 * off-diagonal part vanishes to rounding. */
static void sym3_jacobi(const double A_in[3][3], double vals[3], double Qout[3][3]);
static void sym3_top_eigvec(const double A_in[3][3], double v[3]) {
  double vals[3], Q[3][3];
  sym3_jacobi(A_in, vals, Q);
  int best = 0;
  for (int k = 1; k < 3; ++k)
    if (vals[k] > vals[best]) best = k;
  for (int k = 0; k < 3; ++k) v[k] = Q[k][best];
}

/* all eigenvalues (vals) and eigenvectors (columns of Qout) */
static void sym3_jacobi(const double A_in[3][3], double vals[3], double Qout[3][3]) {
  double A[3][3], Q[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      A[r][c] = A_in[r][c];
      Q[r][c] = r == c ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        /* rotation angle: tan(2 t) = 2 A_pq / (A_qq - A_pp), smaller root */
        double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; ++k) { /* A <- A J (columns p, q) */
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) { /* A <- J^T A (rows p, q) */
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) { /* Q <- Q J */
          double qkp = Q[k][p], qkq = Q[k][q];
          Q[k][p] = c * qkp - sn * qkq;
          Q[k][q] = sn * qkp + c * qkq;
        }
      }
  }
  for (int k = 0; k < 3; ++k) {
    vals[k] = A[k][k];
    for (int c = 0; c < 3; ++c) Qout[k][c] = Q[k][c];
  }
}

/* The maximiser of R over the subgroup: a^T M a is invariant under left
 * multiplication of g by the diagonal phases diag(e^{it}, e^{-it}) of the
 * subgroup (they do not change |U_kk|), which rotate (a0, a3) and (a1, a2)
 * together, so the largest eigenvalue of M is (at least) doubly degenerate
 * and its eigenspace meets a3 = 0. The maximiser is taken there: the top
 * eigenvector of the 3x3 block on (a0, a1, a2), sign fixed by a0 >= 0 (then
 * a1 >= 0, a2 >= 0). Returns -1 if M vanishes. */
static int mag_local_max(const double M[4][4], double a[4]) {
  double B[3][3], v[3];
  double nrm = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      B[r][c] = M[r][c];
      nrm += fabs(M[r][c]);
    }
  if (!(nrm > 1e-300)) return -1;
  sym3_top_eigvec(B, v);
  double sgn = 1.0;
  if (v[0] < 0 || (v[0] == 0 && (v[1] < 0 || (v[1] == 0 && v[2] < 0)))) sgn = -1.0;
  double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  a[0] = sgn * v[0] / n;
  a[1] = sgn * v[1] / n;
  a[2] = sgn * v[2] / n;
  a[3] = 0.0;
  return 0;
}

int or_mag_local_max(const double* U, const int32_t dims[4], int64_t s, int sg, double a[4]) {
  lat_t L = make_lat(dims);
  double M[4][4];
  mag_matrix(U, &L, s, sg, M);
  return mag_local_max(M, a);
}

/* Alg. 1 with the MAG local step: for each subgroup in turn, M from the
 * current links, the maximiser a, its power a^omega (or_overrelax_form), and
 * the 8 links transformed. */
static void mag_site_update(double* U, const lat_t* L, int64_t s, double omega, int form) {
  for (int sg = 0; sg < 3; ++sg) {
    int i = SG_I[sg], j = SG_J[sg];
    double M[4][4], a[4], g[4];
    mag_matrix(U, L, s, sg, M);
    if (mag_local_max(M, a) < 0) continue;
    if (or_overrelax_form(a, omega, form, g) < 0) continue;
    mat3 G = embed_su2(g, i, j);
    mat3 Gd = mat_dag(&G);
    for (int mu = 0; mu < 4; ++mu) {
      int64_t sb = neighbour(L, s, mu, -1);
      mat3 Uf = get_link(U, s, mu);
      mat3 Ub = get_link(U, sb, mu);
      mat3 Ufn = mat_mul(&G, &Uf);
      mat3 Ubn = mat_mul(&Ub, &Gd);
      put_link(U, s, mu, &Ufn);
      put_link(U, sb, mu, &Ubn);
    }
  }
}

int or_mag_sweep(double* U, const int32_t dims[4], int parity, double omega, int form) {
  if (!U || or_check_dims(dims) != 0 || (parity != 0 && parity != 1)) return -1;
  if (!(omega >= 1.0 && omega < 2.0) || form < 0 || form > 3) return -1;
  lat_t L = make_lat(dims);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < L.V; ++s)
    if (site_parity(&L, s) == parity) mag_site_update(U, &L, s, omega, form);
  return 0;
}

/* Relative gaps (l1 - l2) / |l1| between the two largest eigenvalues of the
 * 3x3 block of M that the update of site s (as in or_mag_sweep with omega,
 * form) meets at each of its three subgroup steps, on a copy of the field (0
 * where a step is skipped). A small gap means the maximiser is (nearly) not
 * unique, so that another choice is as good a maximiser. */
int or_mag_site_gaps(const double* U, const int32_t dims[4], int64_t s, double omega, int form,
                     double gaps[3]) {
  if (!U || !gaps || or_check_dims(dims) != 0) return -1;
  lat_t L = make_lat(dims);
  if (s < 0 || s >= L.V) return -1;
  size_t n = (size_t)L.V * 4 * 18;
  double* W = (double*)malloc(n * sizeof(double));
  if (!W) return -1;
  memcpy(W, U, n * sizeof(double));
  for (int sg = 0; sg < 3; ++sg) {
    int i = SG_I[sg], j = SG_J[sg];
    double M[4][4], a[4], g[4], B[3][3], vals[3], Q[3][3];
    gaps[sg] = 0.0;
    mag_matrix(W, &L, s, sg, M);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) B[r][c] = M[r][c];
    sym3_jacobi(B, vals, Q);
    double l1 = fmax(vals[0], fmax(vals[1], vals[2]));
    double l3 = fmin(vals[0], fmin(vals[1], vals[2]));
    double l2 = vals[0] + vals[1] + vals[2] - l1 - l3;
    if (mag_local_max(M, a) < 0) continue;
    gaps[sg] = fabs(l1) > 0 ? (l1 - l2) / fabs(l1) : 0.0;
    if (or_overrelax_form(a, omega, form, g) < 0) continue;
    mat3 G = embed_su2(g, i, j);
    mat3 Gd = mat_dag(&G);
    for (int mu = 0; mu < 4; ++mu) {
      int64_t sb = neighbour(&L, s, mu, -1);
      mat3 Uf = get_link(W, s, mu);
      mat3 Ub = get_link(W, sb, mu);
      mat3 A = mat_mul(&G, &Uf);
      mat3 Bm = mat_mul(&Ub, &Gd);
      put_link(W, s, mu, &A);
      put_link(W, sb, mu, &Bm);
    }
  }
  free(W);
  return 0;
}

/* F_MAG = R / (N_c 4 V): 1 exactly when every link is diagonal. */
double or_mag_functional(const double* U, const int32_t dims[4]) {
  lat_t L = make_lat(dims);
  double* per_site = (double*)malloc(sizeof(double) * (size_t)L.V);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < L.V; ++s) {
    double acc = 0.0;
    for (int mu = 0; mu < 4; ++mu) {
      mat3 A = get_link(U, s, mu);
      for (int k = 0; k < 3; ++k) acc += cx_abs2(A.m[k][k]);
    }
    per_site[s] = acc;
  }
  double sum = 0.0;
  for (int64_t s = 0; s < L.V; ++s) sum += per_site[s];
  free(per_site);
  return sum / (3.0 * 4.0 * (double)L.V);
}

/* theta_MAG = (1 / (N_c V)) sum_x sum_subgroups (M_01^2 + M_02^2): at a = 1 the
 * derivatives of R along the two off-diagonal generators of a subgroup are
 * 2 M_01 and 2 M_02 (the third, diagonal generator is a symmetry, M_03 = 0),
 * so theta_MAG vanishes exactly at stationary points of R. */
double or_mag_theta(const double* U, const int32_t dims[4]) {
  lat_t L = make_lat(dims);
  double* per_site = (double*)malloc(sizeof(double) * (size_t)L.V);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < L.V; ++s) {
    double acc = 0.0;
    for (int sg = 0; sg < 3; ++sg) {
      double M[4][4];
      mag_matrix(U, &L, s, sg, M);
      acc += M[0][1] * M[0][1] + M[0][2] * M[0][2];
    }
    per_site[s] = acc;
  }
  double sum = 0.0;
  for (int64_t s = 0; s < L.V; ++s) sum += per_site[s];
  free(per_site);
  return sum / (3.0 * (double)L.V);
}

/* the while-theta loop of Alg. 1 for the MAG, checks as in or_fix */
int or_fix_mag(double* U, const int32_t dims[4], double omega, int form, double theta_target,
               int32_t max_sweeps, int32_t check_every, int32_t reunit_at_check,
               int32_t* sweeps_out, double* F_out, double* theta_out) {
  if (!U || or_check_dims(dims) != 0 || check_every < 1 || max_sweeps < 0) return -1;
  if (!(omega >= 1.0 && omega < 2.0) || form < 0 || form > 3) return -1;
  int64_t V = or_volume(dims);
  int32_t sweeps = 0;
  int converged = 0;
  double F = 0.0, th = 0.0;
  for (;;) {
    if (sweeps > 0 && reunit_at_check) or_reunitarize(U, V * 4);
    F = or_mag_functional(U, dims);
    th = or_mag_theta(U, dims);
    if (th < theta_target) { converged = 1; break; }
    if (sweeps >= max_sweeps) break;
    for (int32_t k = 0; k < check_every && sweeps < max_sweeps; ++k) {
      or_mag_sweep(U, dims, 0, omega, form);
      or_mag_sweep(U, dims, 1, omega, form);
      ++sweeps;
    }
  }
  if (sweeps_out) *sweeps_out = sweeps;
  if (F_out) *F_out = F;
  if (theta_out) *theta_out = th;
  return converged ? 0 : 1;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
