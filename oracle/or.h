/*
 * or.h -- plain FP64 CPU oracle for checkerboard overrelaxation gauge fixing
 * (Schroeck & Vogt, "Gauge fixing using overrelaxation and simulated annealing
 * on GPUs", arXiv:1209.4008).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark call this library. The GPU library shares no
 * code with it, and no product code path may route through it.
 *
 * Field layout (canonical, host memory): complex128, interleaved (re, im),
 *   U[s][mu][a][b]  with  s = ((t*nz + z)*ny + y)*nx + x,
 * i.e. double index ((s*4 + mu)*9 + 3*a + b)*2 + {0: re, 1: im}.
 * dims = {nt, nz, ny, nx}; direction mu = 0 is t, mu = 1, 2, 3 are x, y, z.
 * Boundaries are periodic; every extent must be even and >= 2 so that the
 * two checkerboard sublattices share no link (Sec. 2, RED/BLACK
 * decomposition). Parity of a site is (t + x + y + z) mod 2; RED = 0.
 *
 * Gauge: OR_LANDAU sums directions mu = 0..3 in K(x), F and theta;
 * OR_COULOMB sums mu = 1..3 only and reports F and theta per timeslice.
 * In both gauges the site transformation is applied to all four links
 * U_mu(x) and U_mu(x - mu) (the temporal links of the Coulomb gauge are
 * transformed in place so that the output is a gauge transform of the input).
 *
 * Functions returning int return 0 on success and a negative value on bad
 * arguments (odd or too small extents, omega outside [1, 2), T <= 0).
 */
#ifndef GF_ORACLE_OR_H
#define GF_ORACLE_OR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_LANDAU 0
#define OR_COULOMB 1

/* geometry ---------------------------------------------------------------- */
int     or_check_dims(const int32_t dims[4]);
int64_t or_volume(const int32_t dims[4]);
int     or_num_threads(void);
void    or_set_num_threads(int n);

/* building blocks (exposed so that the tests can pin each step) ----------- */
/* Quaternion (a0, a1, a2, a3) <-> SU(2) matrix [[a0+i a3, a2+i a1],
 * [-a2+i a1, a0-i a3]].  Given a 3x3 complex M (18 doubles, row major) and a
 * subgroup (i, j), q receives the quaternion (SU(2)-proportional) part of the
 * 2x2 block M[{i,j},{i,j}]. */
void or_su2_part(const double M[18], int i, int j, double q[4]);
/* Overrelaxed local transformation s = g^omega from the unnormalised
 * quaternion q of K^dagger (Sec. 2, overrelaxation paragraph; the form is the
 * reading documented at the definition): unit norm on output. Returns -1 if
 * |q| is degenerate. */
int  or_overrelax(const double q[4], double omega, double s[4]);
/* The other forms of g^omega (Sec. 2, overrelaxation paragraph: the power is
 * taken to first or second order): with g = q/|q| = 1 + a, form 1 is
 * 1 + omega a, form 2 is 1 + omega a + omega (omega-1)/2 a^2 (both projected
 * onto SU(2) by normalising), form 3 the exact power (cos(omega phi),
 * n sin(omega phi)) of g = (cos phi, n sin phi); form 0 is or_overrelax.
 * Unit norm on output. Returns -1 for a degenerate q or an invalid form. */
int  or_overrelax_form(const double q[4], double omega, int form, double s[4]);
/* K(x) of eq. (5) (sum over mu of U_mu(x) + U_mu(x-mu)^dagger) at site s. */
void or_local_K(const double* U, const int32_t dims[4], int gauge, int64_t s, double K[18]);

/* the hot path ------------------------------------------------------------ */
/* One checkerboard half-sweep of overrelaxation over the sites of one parity
 * (Sec. 2, Alg. 1; omega = 1 is plain relaxation). */
int  or_sweep(double* U, const int32_t dims[4], int gauge, int parity, double omega);
/* The same half-sweep with the power g^omega taken in the given form
 * (or_overrelax_form; form 0 is or_sweep). */
int  or_sweep_form(double* U, const int32_t dims[4], int gauge, int parity, double omega,
                   int form);
/* The same update on a list of sites of one parity only (sampled checks). */
int  or_update_sites(double* U, const int32_t dims[4], int gauge, double omega,
                     const int64_t* sites, int64_t n);
/* The annealing heatbath update on a list of sites of one parity only. */
int  or_heatbath_sites(double* U, const int32_t dims[4], int gauge, double T, uint64_t seed,
                       uint64_t sweep, const int64_t* sites, int64_t n);
/* Gauge functional eq. (3), normalised so that U = 1 gives 1. out[0] (Landau)
 * or out[t], t < nt (Coulomb). Returns the Landau value or the mean over t. */
double or_functional(const double* U, const int32_t dims[4], int gauge, double* out);
/* Raw (unnormalised) sum Re sum_{x,mu in D} tr U_mu(x) of eq. (3). */
double or_functional_raw(const double* U, const int32_t dims[4], int gauge);
/* Precision theta of Sec. 2 computed from the lattice gauge potential A_mu
 * (theta_A) and from the local sums K(x) (theta_K); same output convention as
 * or_functional; the return value is the Landau value or the max over t. */
double or_theta_A(const double* U, const int32_t dims[4], int gauge, double* out);
double or_theta_K(const double* U, const int32_t dims[4], int gauge, double* out);
/* Gram-Schmidt projection of each link back onto SU(3). */
void   or_reunitarize(double* U, int64_t n_links);
/* Unitarity deviation: max over links and elements of |(U U^dag - 1)_ab|;
 * +Inf if a link holds a NaN. */
double or_unitarity(const double* U, const int32_t dims[4]);
/* Average plaquette (1/3) Re tr of the elementary plaquette. */
double or_plaquette(const double* U, const int32_t dims[4]);
/* U_mu(x) <- g(x) U_mu(x) g(x+mu)^dagger, g[s][3][3] complex128 (eq. (4)). */
int    or_gauge_transform(double* U, const int32_t dims[4], const double* g);

/* Driver: sweeps (RED then BLACK, g^omega in the given form) with a check
 * every check_every sweeps, starting before the first sweep; at each check
 * after the first, the field is first reunitarised if reunit_at_check != 0.
 * Stops when theta < target (Coulomb: max over timeslices) or when
 * max_sweeps is reached. Returns 0 if converged, 1 if not, <0 on bad
 * arguments. */
int or_fix(double* U, const int32_t dims[4], int gauge, double omega, int form,
           double theta_target, int32_t max_sweeps, int32_t check_every,
           int32_t reunit_at_check, int32_t* sweeps_out, double* F_out,
           double* theta_out);

/* Coulomb gauge (Sec. 1) with each timeslice frozen (no longer swept) from
 * the first check at which its theta_t is below the target; the timeslices
 * are independent problems (a driver the paper does not describe). F_out, theta_out: nt values each; frozen_at (or NULL):
 * per timeslice the sweep count at which it was frozen, -1 if never.
 * Returns 0 when every timeslice is frozen, 1 at max_sweeps, <0 on bad
 * arguments. */
int    or_fix_coulomb_frozen(double* U, const int32_t dims[4], double omega, double theta_target,
                             int32_t max_sweeps, int32_t check_every, int32_t reunit_at_check,
                             int32_t* sweeps_out, double* F_out, double* theta_out,
                             int32_t* frozen_at);

/* maximally Abelian gauge (named in Sec. 1 and the summary, functional from
 * the literature): maximise R = sum_{x,mu} sum_k |U_mu(x)_kk|^2 -------------- */
/* M (4x4, row major) of the quadratic form R_x(a) = a^T M a + const of the 8
 * links at site s under the local transformation embed(a) on subgroup sg
 * ((0,1), (0,2), (1,2)), by polarisation of R evaluated with full products. */
void   or_mag_matrix(const double* U, const int32_t dims[4], int64_t s, int sg, double M[16]);
/* The maximiser of R_x over the subgroup: top eigenvector of M restricted to
 * a3 = 0 (the top eigenvalue is degenerate along the diagonal-phase symmetry),
 * unit norm, a0 >= 0. Returns -1 if M vanishes. */
int    or_mag_local_max(const double* U, const int32_t dims[4], int64_t s, int sg, double a[4]);
/* One checkerboard half-sweep of MAG overrelaxation (maximiser raised to
 * omega in the given form, or_overrelax_form). */
int    or_mag_sweep(double* U, const int32_t dims[4], int parity, double omega, int form);
/* Relative gaps (l1 - l2)/|l1| between the two largest eigenvalues of the
 * 3x3 block of M met at each of the three subgroup steps of the update of
 * site s (as in or_mag_sweep with omega, form), on a copy of the field; 0 for
 * a skipped step. A small gap: the maximiser is (nearly) not unique. */
int    or_mag_site_gaps(const double* U, const int32_t dims[4], int64_t s, double omega,
                        int form, double gaps[3]);
/* F_MAG = R / (3 * 4 V) (1 when all links are diagonal). */
double or_mag_functional(const double* U, const int32_t dims[4]);
/* theta_MAG = (1/(3V)) sum_x sum_sg (M_01^2 + M_02^2): the squared gradient of
 * R along the six off-diagonal generators, 0 at stationary points. */
double or_mag_theta(const double* U, const int32_t dims[4]);
/* Driver as or_fix, with the MAG sweep, functional and theta. */
int    or_fix_mag(double* U, const int32_t dims[4], double omega, int form, double theta_target,
                  int32_t max_sweeps, int32_t check_every, int32_t reunit_at_check,
                  int32_t* sweeps_out, double* F_out, double* theta_out);

/* simulated annealing ----------------------------------------------------- */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Kennedy-Pendleton draw of X0 with density ~ sqrt(1-X0^2) exp(alpha X0),
 * using the same Philox streams as the annealing sweep for (site, sweep,
 * subgroup). Returns the number of attempts used (0 if the cap was hit). */
int  or_kp_draw(double alpha, uint64_t seed, uint64_t site, uint64_t sweep,
                int subgroup, double* X0);
/* Full SU(2) draw X (X0 as above, direction uniform) for the same streams. */
int  or_heatbath_su2(double alpha, uint64_t seed, uint64_t site, uint64_t sweep,
                     int subgroup, double X[4]);
/* Stochastic relaxation half-sweep (Sec. 1): for each site and subgroup,
 * with probability prob (Philox draw keyed by seed, counter (site, sweep,
 * 0x1200 | subgroup, 0), first uniform) the microcanonical step g = ghat^2,
 * otherwise the overrelaxation step with omega (omega = 1: relaxation). */
int  or_sweep_sr(double* U, const int32_t dims[4], int gauge, int parity, double omega,
                 double prob, uint64_t seed, uint64_t sweep);
/* Heatbath half-sweep of the annealing step at temperature T: the local
 * transformation is drawn with weight exp(Re tr[g K] / T). n_capped (may be
 * NULL) accumulates the number of subgroup updates that hit the attempt cap. */
int  or_heatbath_half(double* U, const int32_t dims[4], int gauge, int parity,
                      double T, uint64_t seed, uint64_t sweep, int64_t* n_capped);
/* Microcanonical half-sweep: g = (local maximum)^2, which leaves Re tr[g K]
 * unchanged. */
/* A half-sweep of one of the updates above (kind 0 overrelaxation with omega,
 * 1 heatbath at temperature param, 2 microcanonical, 3 stochastic relaxation
 * with probability param; seed and sweep key the draws) that also writes
 * g[s] (V x 3 x 3 complex128): each updated site's total transformation, the
 * product of its three subgroup factors; 1 at the sites of the other parity. */
int  or_half_sweep_g(double* U, const int32_t dims[4], int gauge, int parity, int kind,
                     double omega, double param, uint64_t seed, uint64_t sweep, double* g);
/* Every result the heatbath update of site s (as in or_heatbath_half with T,
 * seed, sweep) can have when each Kennedy-Pendleton trial whose accept margin
 * |(1 - lambda^2) - u4^2| is below tau may be decided either way, as a
 * sampler in lower precision may decide it. Outcome 0 is the exact result;
 * the others are explored depth first, each deciding one more borderline
 * trial the other way. An outcome is the 8 links the update moves, U_mu(s),
 * mu = 0..3, then U_mu(s - mu), 18 doubles each, into links_out
 * (max_out x 8 x 18). min_margin (may be NULL) receives the smallest margin
 * met on the exact path. Returns the number of outcomes (<= max_out) or -1.
 * The field is not changed. */
int  or_heatbath_site_outcomes(const double* U, const int32_t dims[4], int gauge, double T,
                               uint64_t seed, uint64_t sweep, int64_t s, double tau,
                               int max_out, double* links_out, double* min_margin);
int  or_micro_half(double* U, const int32_t dims[4], int gauge, int parity);
/* One annealing step: heatbath RED, BLACK, then n_micro microcanonical
 * sweeps (RED, BLACK each). */
int  or_anneal_sweep(double* U, const int32_t dims[4], int gauge, double T,
                     uint64_t seed, uint64_t sweep, int n_micro, int64_t* n_capped);

#ifdef __cplusplus
}
#endif
#endif
