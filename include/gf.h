/*
 * gf.h -- C ABI of libgf, an MI355X (gfx950) implementation of checkerboard
 * overrelaxation gauge fixing with simulated-annealing preconditioning
 * (Schroeck & Vogt, "Gauge fixing using overrelaxation and simulated
 * annealing on GPUs", arXiv:1209.4008).
 *
 * Conventions used by every call
 * ------------------------------
 * Lattice: periodic, extents (nt, nz, ny, nx), each even and >= 2 (the
 *   RED/BLACK decomposition of Sec. 2 needs even extents so that the sites of
 *   one colour share no link), V = nt*nz*ny*nx <= 2^30. Direction mu = 0 is t,
 *   mu = 1, 2, 3 are x, y, z. Canonical site index
 *   s = ((t*nz + z)*ny + y)*nx + x; parity (t+x+y+z) mod 2, RED = 0.
 * Canonical field (host or device, caller's choice where stated):
 *   complex128 U[s][mu][a][b], i.e. 18 doubles per link, rows a, columns b.
 * Device field (the layout every sweep works on, Sec. 4.1: the gauge field
 *   is split into a RED and a BLACK block and the site index runs fastest):
 *   complex elements of the precision `prec` (float2 or double2),
 *     elem(p, mu, c, h) at offset
 *       p*4*NC*Vp + (h/2048)*2048*4*NC + (mu*NC + c)*2048 + h%2048,
 *   p = parity, h = s >> 1 (the half index), c = 3a + b < NC,
 *   NC = storage/2: 9 complex (18 reals) or 6 complex (12 reals: rows 0 and 1;
 *   row 2 is rebuilt as conj(row0 x row1), Sec. 4.1), Vp = V/2 rounded up to
 *   a multiple of 2048. That is, the sites of each parity are cut into tiles
 *   of 2048 consecutive half indices; a tile holds its links direction after
 *   direction and component after component, the site index running fastest.
 *   Elements of the padding sites h >= V/2 are never read. Size:
 *   gf_field_bytes() = 8 Vp storage prec bytes.
 * Gauge: GF_LANDAU uses mu = 0..3 in K(x), F and theta (eq. (3), (5), (7));
 *   GF_COULOMB uses the spatial mu = 1..3 and reports F and theta per
 *   timeslice (arrays of nt doubles). GF_MAG, the maximally Abelian gauge
 *   (named in Sec. 1; the paper does not write out its functional), maximises
 *   R = sum_{x,mu} sum_k |U_mu(x)_kk|^2: in each SU(2) subgroup the site's R is
 *   a quadratic form a^T M a in the quaternion a of the local transformation,
 *   maximised by the top eigenvector of M restricted to a3 = 0 (the subgroup's
 *   diagonal phases are a symmetry); F = R / (12 V) (1 iff all links are
 *   diagonal), theta = sum_x sum_subgroups (M01^2 + M02^2) / (3 V) (the squared
 *   gradient along the off-diagonal generators). In all gauges each site
 *   transformation is applied to all 8 links at the site, so the result is a
 *   gauge transform of the input.
 *
 * Memory and streams: every pointer passed to a compute call is device memory
 * owned by the caller; the library never frees it. Calls enqueue work on the
 * context stream and return without waiting, except gf_fix, gf_fix_mixed,
 * gf_batch_run and the *_host helpers, which synchronise that stream.
 * A context is used by one host thread at a time.
 *
 * Errors: every call returns a gf_status. Arguments are validated on the host
 * before anything is enqueued, so a call that returns an error has not
 * touched device memory. gf_last_error() holds a message for the last failure
 * on a context.
 */
#ifndef GF_H
#define GF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gf_status;
#define GF_OK 0
#define GF_NOT_CONVERGED 1     /* driver stopped at max_sweeps (information) */
#define GF_ERR_ARG (-1)        /* invalid argument (nothing enqueued)        */
#define GF_ERR_UNSUPPORTED (-2)
#define GF_ERR_DEVICE (-3)     /* no usable GPU                              */
#define GF_ERR_HIP (-4)        /* HIP runtime error                          */
#define GF_ERR_NONFINITE (-5)  /* F or theta became NaN or Inf               */
#define GF_ERR_NOMEM (-6)

#define GF_LANDAU 0
#define GF_COULOMB 1
#define GF_MAG 2   /* overrelaxation sweeps, measurement and the drivers only */
#define GF_FP32 4
#define GF_FP64 8
#define GF_R12 12
#define GF_R18 18

typedef struct {
  int32_t nt, nz, ny, nx; /* even, >= 2 */
  int32_t prec;           /* GF_FP32 | GF_FP64 */
  int32_t storage;        /* GF_R12 | GF_R18   */
} gf_geom;

typedef struct gf_ctx gf_ctx;

/* ---- context and host-only helpers -------------------------------------- */
/* Create a context on `device` enqueuing on `hip_stream` (a hipStream_t; NULL
 * = the default stream). Fails with GF_ERR_DEVICE when no GPU is present. */
gf_status gf_create(int device, void* hip_stream, gf_ctx** out);
gf_status gf_destroy(gf_ctx* ctx);
/* Message for the last failure on ctx, or for the last failed gf_create when
 * ctx is NULL. Never NULL. */
const char* gf_last_error(const gf_ctx* ctx);
/* Host-only: GF_OK if geom is valid, GF_ERR_ARG otherwise. */
gf_status gf_check_geom(const gf_geom* geom);
/* Host-only: bytes of a device field, 8 Vp storage prec (Vp = V/2 rounded up
 * to a multiple of 2048); 0 if geom invalid. */
size_t gf_field_bytes(const gf_geom* geom);
/* Host-only: runs the library's host-side self checks (index arithmetic);
 * GF_OK when they pass. */
gf_status gf_selftest_host(void);
/* Library version string. */
const char* gf_version(void);

/* ---- layout (Sec. 4.1: RED/BLACK blocks, site index fastest, 12 reals) --- */
/* Canonical FP64 field in device memory -> device field of geom's precision
 * and storage (rounded to nearest for FP32; row 2 dropped for R12). */
gf_status gf_pack(gf_ctx* ctx, const gf_geom* geom, const double* U_canon_dev, void* U_dev);
/* Device field -> canonical FP64 field in device memory (row 2 rebuilt in
 * FP64 for R12). */
gf_status gf_unpack(gf_ctx* ctx, const gf_geom* geom, const void* U_dev, double* U_canon_dev);
/* Device field -> device field of another precision/storage (same extents).
 * With reunitarize != 0 each link is projected onto SU(3) by Gram-Schmidt in
 * FP64 on the way. Source and destination must not overlap. */
gf_status gf_convert(gf_ctx* ctx, const gf_geom* src, const void* U_src, const gf_geom* dst,
                     void* U_dst, int32_t reunitarize);

/* ---- the hot path ----------------------------------------------------------- */
/* One checkerboard half-sweep of overrelaxation (Alg. 1) over the sites of
 * `parity`: per site, K(x) of eq. (5) from its 8 links, then for the SU(2)
 * subgroups (0,1), (0,2), (1,2) in turn the local maximum of eq. (6) raised to
 * the power omega (Sec. 2; the 19-flop form s = (c r0, b c r) with
 * b = (omega r0^2 + |r|^2)/(r0^2 + |r|^2), c = (r0^2 + b^2 |r|^2)^(-1/2)),
 * and the product transformation applied to the 8 links in place. With 12-real
 * storage the two stored rows of each updated forward link are then
 * re-orthonormalised by Gram-Schmidt (in an FP32 field with the squared norms
 * summed in FP64 and one rounding per element, which keeps the field on its
 * gauge orbit). omega in [1, 2) (1 = plain relaxation); otherwise GF_ERR_ARG. */
gf_status gf_sweep(gf_ctx* ctx, void* U, const gf_geom* geom, int32_t gauge, int32_t parity,
                   double omega);
/* gf_sweep with another form of the power g^omega (Sec. 2: the power is taken
 * to first or second order). With g = q/|q| = 1 + a the local maximum:
 * form 1: 1 + omega a; form 2: 1 + omega a + omega (omega - 1)/2 a^2; form 3:
 * the exact power (cos(omega phi), n sin(omega phi)) of g = (cos phi, n sin phi)
 * (left at g when g has no axis); each divided by its length. form 0 is
 * gf_sweep. omega in [1, 2), form in 0..3; otherwise GF_ERR_ARG. */
gf_status gf_sweep_form(gf_ctx* ctx, void* U, const gf_geom* geom, int32_t gauge, int32_t parity,
                        double omega, int32_t form);
/* Stochastic relaxation half-sweep (Sec. 1): as gf_sweep, but for each site
 * and subgroup, with probability prob in [0, 1] the microcanonical step
 * g = ghat^2 replaces the overrelaxation step. Draw: Philox4x32-10, key (seed
 * low, seed high), counter (site, sweep, 0x1200 | subgroup, 0), first
 * uniform (u + 1/2) 2^-32 < prob. prob = 0 is gf_sweep. */
gf_status gf_sweep_sr(gf_ctx* ctx, void* U, const gf_geom* geom, int32_t gauge, int32_t parity,
                      double omega, double prob, uint64_t seed, uint64_t sweep);
/* Gauge functional eq. (3), normalised so that the unit field gives 1:
 * F = Re sum_{x, mu in D} tr U_mu(x) / (3 |D| V) (Landau, F_dev[0]) or per
 * timeslice / (9 V_s) (Coulomb, F_dev[0..nt-1]). Accumulated in FP64. */
gf_status gf_functional(gf_ctx* ctx, const void* U, const gf_geom* geom, int32_t gauge,
                        double* F_dev);
/* Precision theta of eq. (7): theta = sum_x tr[Delta(x) Delta(x)^dag] / (3 V)
 * with Delta(x) = sum_{mu in D} [A_mu(x) - A_mu(x - mu)], A_mu the traceless
 * part of (U_mu - U_mu^dag)/(2i) (theta_dev[0], Landau) or per timeslice with
 * V -> V_s (Coulomb, theta_dev[0..nt-1]). Accumulated in FP64. */
gf_status gf_theta(gf_ctx* ctx, const void* U, const gf_geom* geom, int32_t gauge,
                   double* theta_dev);
/* F and theta in one pass over the field (what the drivers use). */
gf_status gf_measure(gf_ctx* ctx, const void* U, const gf_geom* geom, int32_t gauge,
                     double* F_dev, double* theta_dev);
/* gf_measure for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, with the per-block partial sums in a fixed 4 MiB
 * device array of the library (one per GPU, set up by gf_create, kept until
 * the process ends) instead of context memory that gf_measure may allocate.
 * Allocates nothing. Lattices needing more than 2^19 partial sums
 * (2 * ceil(V / (2 nt 256)) * nt; about 2^27 sites) are rejected with
 * GF_ERR_ARG. All calls on one GPU share the array: calls that overlap in time
 * on one GPU (several streams or threads) race and must be serialised by the
 * caller. */
gf_status gf_measure_static(gf_ctx* ctx, const void* U, const gf_geom* geom, int32_t gauge,
                            double* F_dev, double* theta_dev);
/* Project every link onto SU(3) by Gram-Schmidt in FP64 (rows 0, 1
 * orthonormalised; row 2 = conj(row0 x row1) for R18). */
gf_status gf_reunitarize(gf_ctx* ctx, void* U, const gf_geom* geom);
/* Average plaquette (1/(6V)) sum Re tr U_P / 3, in FP64 (support: gauge
 * invariant, so unchanged by every sweep). */
gf_status gf_plaquette(gf_ctx* ctx, const void* U, const gf_geom* geom, double* P_dev);

/* ---- simulated annealing (Sec. 1: preconditioner) ------------------------- */
/* Heatbath half-sweep at temperature T > 0: per site and subgroup the SU(2)
 * transformation is drawn with weight exp(Re tr[g K(x)] / T) (Kennedy-
 * Pendleton, Philox4x32-10 keyed by seed, counter (site, sweep, tag,
 * attempt); up to 1024 attempts, after which the subgroup is left unchanged). */
gf_status gf_heatbath_half(gf_ctx* ctx, void* U, const gf_geom* geom, int32_t gauge,
                           int32_t parity, double T, uint64_t seed, uint64_t sweep);
/* Microcanonical half-sweep: g = (local maximum)^2, Re tr[g K] unchanged. */
gf_status gf_micro_half(gf_ctx* ctx, void* U, const gf_geom* geom, int32_t gauge,
                        int32_t parity);
/* One annealing step: heatbath RED and BLACK at T, then n_micro
 * microcanonical sweeps (RED, BLACK each). */
gf_status gf_anneal_sweep(gf_ctx* ctx, void* U, const gf_geom* geom, int32_t gauge, double T,
                          uint64_t seed, uint64_t sweep, int32_t n_micro);
/* Philox4x32-10 of n counters (4 x u32 each, device) with key (seed low,
 * seed high), into out (4 x u32 each, device). Support: the same generator
 * the heatbath uses. */
gf_status gf_philox(gf_ctx* ctx, const uint32_t* ctr_dev, uint64_t seed, uint32_t* out_dev,
                    int64_t n);

/* ---- FP32 updates that track the site transformation ---------------------- */
/* The gauge-transformation field that the FP32 phase of gf_fix_mixed
 * accumulates (Sec. 1, eq. (4): the result of a gauge fixing is the input
 * transformed by one g(x) per site): FP32, rows 0 and 1 of g(x) (row 2 =
 * conj(row0 x row1)), tiled like a 12-real device field with one direction:
 *   elem(p, c, h) at offset p*6*Vp + (h/2048)*2048*6 + c*2048 + h%2048, c = 3a + b.
 * Host-only: its size in bytes, 96 Vp; 0 if geom is invalid. */
size_t gf_gauge_bytes(const gf_geom* geom);
/* G <- 1 at every site (the padding sites included). */
gf_status gf_gauge_unit(gf_ctx* ctx, const gf_geom* geom, void* G);
/* Canonical complex128 g[s][a][b] in device memory (9 complex per site, an
 * SU(3) matrix each) -> G (rows 0 and 1 rounded to FP32; row 2 is implied). */
gf_status gf_gauge_pack(gf_ctx* ctx, const gf_geom* geom, const double* g_canon_dev, void* G);
/* G -> canonical complex128 g[s][a][b] (9 complex per site, row 2 rebuilt in
 * FP64) in device memory. */
gf_status gf_gauge_unpack(gf_ctx* ctx, const gf_geom* geom, const void* G, double* g_canon_dev);
/* gf_sweep, gf_heatbath_half and gf_micro_half on an FP32 field that also
 * accumulate each updated site's whole transformation Gtot (the product of
 * its three subgroup factors) into G: g(x) <- Gtot g(x), rows 0 and 1 then
 * re-orthonormalised as 12-real FP32 links are (gf_sweep). Starting from G = 1, any sequence of such calls
 * leaves U equal to the input transformed by G (eq. (4)), up to FP32
 * rounding. geom must be FP32 (else GF_ERR_UNSUPPORTED); G (gf_gauge_bytes of
 * geom) must not overlap U. The heatbath and microcanonical calls reject
 * GF_MAG; gf_sweep_tracked takes all gauges. */
gf_status gf_sweep_tracked(gf_ctx* ctx, void* U, void* G, const gf_geom* geom, int32_t gauge,
                           int32_t parity, double omega);
gf_status gf_heatbath_half_tracked(gf_ctx* ctx, void* U, void* G, const gf_geom* geom,
                                   int32_t gauge, int32_t parity, double T, uint64_t seed,
                                   uint64_t sweep);
gf_status gf_micro_half_tracked(gf_ctx* ctx, void* U, void* G, const gf_geom* geom,
                                int32_t gauge, int32_t parity);

/* ---- tuning --------------------------------------------------------------- */
/* Variant of the sweep kernels for one (precision, storage) pair on this
 * context: tps = lanes per site (1, 2 or 4; with k lanes each lane owns the
 * forward and backward links of 4/k directions and the lanes add their parts
 * of K(x)), nontemporal = 0 for ordinary link accesses, 1 to mark the link
 * loads and stores as streaming, 2 to stream the stores only (loads cached;
 * pays when the cache holds part of the field between half-sweeps; the
 * overrelaxation and stochastic-relaxation sweeps, the annealing updates run
 * 2 as 1). The context keeps two tables: the overrelaxation sweeps (every
 * form, stochastic relaxation, GF_MAG; gf_set_sweep_variant) and the
 * annealing updates (heatbath and microcanonical; gf_set_anneal_variant),
 * each per (precision, storage) and per size class (fields of at most 2 GiB,
 * larger ones). These calls set both size classes; the autotuners set the
 * class of the field they time.
 * tps = 0 / nontemporal = -1 restore the built-in defaults: for FP64 4 lanes,
 * except 1 lane for the sweeps over more than 2 GiB of fields; for FP32 2
 * lanes (sweeps) and 1 lane (annealing); nontemporal 0 for fields of at most
 * 2 GiB (the Infinity Cache then serves part of every half-sweep), 1 for
 * larger ones. */
gf_status gf_set_sweep_variant(gf_ctx* ctx, int32_t prec, int32_t storage, int32_t tps,
                               int32_t nontemporal);
gf_status gf_set_anneal_variant(gf_ctx* ctx, int32_t prec, int32_t storage, int32_t tps,
                                int32_t nontemporal);
/* The sweep variant for (prec, storage) and a field of at most 2 GiB. */
gf_status gf_get_sweep_variant(gf_ctx* ctx, int32_t prec, int32_t storage, int32_t* tps,
                               int32_t* nontemporal);
/* The variant the sweeps (resp. the annealing updates) of `geom`'s field use
 * on this context: the set or tuned one of its size class, else the built-in
 * one. */
gf_status gf_sweep_variant_for(gf_ctx* ctx, const gf_geom* geom, int32_t* tps,
                               int32_t* nontemporal);
gf_status gf_anneal_variant_for(gf_ctx* ctx, const gf_geom* geom, int32_t* tps,
                                int32_t* nontemporal);
/* Autotuner of the overrelaxation sweep for geom (its extents, precision and
 * storage): on a scratch field (allocated and freed inside the call) that
 * starts as a copy of U_like (a device field of geom; NULL: the unit field),
 * each of the nine variants (tps 1, 2, 4) x (nontemporal 0, 1, 2) runs a
 * block of RED/BLACK sweep pairs (omega 1.7) captured as a hipGraph, as the
 * drivers replay theirs (100 sweeps, the drivers' check interval, or about
 * 100 ms of work for large fields); the nine blocks are
 * replayed in turn for five rounds and each variant's time is the median of
 * its rounds. The fastest is kept on this context for geom's precision,
 * storage and size class, and returned. The caller's fields are not modified.
 * ms_out (NULL or 9 floats, index 3*nontemporal + log2(tps)) receives the
 * time per half-sweep of each. Synchronises the context stream. */
gf_status gf_autotune(gf_ctx* ctx, const gf_geom* geom, int32_t gauge, const void* U_like,
                      int32_t* tps_out, int32_t* nt_out, float* ms_out);
/* The same for the annealing updates (GF_LANDAU or GF_COULOMB): the unit of
 * work is one annealing step at temperature T (heatbath RED and BLACK, one
 * microcanonical sweep, the same draws in every replay); ms_out per
 * half-sweep. */
gf_status gf_autotune_anneal(gf_ctx* ctx, const gf_geom* geom, int32_t gauge, const void* U_like,
                             double T, int32_t* tps_out, int32_t* nt_out, float* ms_out);
/* Storage axis: packs the canonical FP64 field U_canon (device) into scratch
 * fields of geom's extents and precision in 12 and 18 reals, tunes the sweep
 * variants of each (gf_autotune, which keeps each one's best on the context)
 * and returns in *storage_out the storage whose best variant sweeps the
 * lattice fastest (GF_R12 or GF_R18); ms_out (NULL or 2 floats): the best
 * time per half-sweep of each. geom->storage is ignored. */
gf_status gf_autotune_storage(gf_ctx* ctx, const gf_geom* geom, int32_t gauge,
                              const double* U_canon, int32_t* storage_out, float* ms_out);

/* Bandwidth probe (measurement support): streams `bytes` (a multiple of 16)
 * with 16-byte accesses, one per thread. kind 0: copy src -> dst; kind 1:
 * in-place nontemporal read-modify-write of dst (dst[i] = 2 dst[i]); kind 2:
 * read src only (one partial sum per 256 elements is written to dst, which
 * must hold bytes/2048 doubles). Enqueued on the context
 * stream; time it with events around the call. */
gf_status gf_stream_probe(gf_ctx* ctx, const void* src, void* dst, size_t bytes, int32_t kind);

/* Unitarity monitor: into dev_out (device, 1 double) the largest
 * |(U U^dag)_ab - delta_ab| over all links and elements (row 2 of 12-real
 * links rebuilt first, everything in FP64); +Inf if any link holds a NaN.
 * SU(3) links give 0 up to rounding; the rounding of the updates makes it
 * grow between the drivers' reunitarisations, which remove it. Uses the
 * context's partial-sum buffer. */
gf_status gf_unitarity(gf_ctx* ctx, const void* U, const gf_geom* geom, double* dev_out);

/* ---- drivers (the while-theta loop of Alg. 1) ------------------------------- */
#define GF_FLAG_TIMING 1u    /* record hipEvent kernel timings into the result */
#define GF_FLAG_GRAPH 2u     /* replay the sweeps between checks as a hipGraph */
#define GF_FLAG_NO_TRACK 4u  /* gf_fix_mixed: do not track g in the FP32 phase   */
/* GF_COULOMB only (else GF_ERR_ARG; batches GF_ERR_UNSUPPORTED): freeze each
 * timeslice from the first check at which its theta_t < the phase's target
 * on (its sites are no longer updated; reunitarisation still covers the
 * whole field); a phase ends when every timeslice is frozen. Coulomb gauge
 * (Sec. 1: the condition on the spatial components only) is one independent
 * problem per timeslice: F and theta_t involve the spatial links of
 * timeslice t only, and a site update changes the spatial links of its own
 * timeslice only, so the frozen timeslices keep the theta_t they converged
 * with, and the sweeps go to the ones that have not. */
#define GF_FLAG_FREEZE_TIMESLICES 8u
/* At every check, before its reunitarisation, measure the field's unitarity
 * deviation (gf_unitarity): the drift that the sweeps since the previous
 * check left in the links. Reported in gf_fix_result.unitarity_max and, per
 * check, in the check log. Not used by gf_batch_run. */
#define GF_FLAG_MONITOR 16u

/* One check of gf_fix or gf_fix_mixed, written to params.check_log. */
typedef struct {
  int32_t sweeps;          /* sweeps of the phase before this check                */
  int32_t prec;            /* GF_FP32 or GF_FP64: the field checked                */
  double F, theta;         /* as in gf_fix_result (Coulomb: mean F, max theta)     */
  double unitarity;        /* GF_FLAG_MONITOR: the field's unitarity deviation
                              before the check's reunitarisation; else -1          */
  double elapsed_ms;       /* host time since the call started                     */
} gf_check_record;

typedef struct {
  double omega;            /* overrelaxation parameter, [1, 2)                         */
  double theta_target;     /* stop when theta (Coulomb: max over t) < theta_target     */
  double theta_switch;     /* gf_fix_mixed: leave the FP32 phase when theta < this     */
  int32_t max_sweeps;      /* per phase                                                */
  int32_t check_every;     /* sweeps between checks (Sec. 4.1 uses 100)                */
  int32_t reunit_at_check; /* reunitarise before every check after the first           */
  uint32_t flags;          /* GF_FLAG_*                                                */
  /* simulated annealing before the overrelaxation (Sec. 1: a preconditioner
   * that raises the chance of reaching the global maximum of F) */
  int32_t sa_steps;        /* 0: none; else steps k = 0..sa_steps-1 of gf_anneal_sweep */
  int32_t sa_micro;        /* microcanonical sweeps per step                           */
  int32_t sa_reunit_every; /* reunitarise after every this many steps (0: never)       */
  int32_t or_form;         /* form of g^omega in the overrelaxation sweeps (gf_sweep_form):
                              0 = the 19-flop form of gf_sweep (default), 1 = first order,
                              2 = second order, 3 = exact; not with sr_prob > 0 and not in
                              batches (GF_ERR_UNSUPPORTED)                               */
  double sa_T0, sa_T1;     /* linear schedule T_k = T0 + (T1 - T0) k / (sa_steps - 1)  */
  uint64_t seed;           /* Philox key of the heatbath draws (sweep index = k)       */
  /* stochastic relaxation instead of plain overrelaxation (Sec. 1): > 0 uses
   * gf_sweep_sr with this probability, sweep index = sweeps of the phase, key
   * = seed; the sweeps are then launched one by one (no graph replay) */
  double sr_prob;
  /* optional host array of check_log_cap records: the drivers write one per
   * check, in order, until it is full (gf_fix_result.check_log_n counts them;
   * NULL: no log). Not used by gf_batch_run. */
  gf_check_record* check_log;
  int32_t check_log_cap;
} gf_fix_params;

typedef struct {
  int32_t status;          /* GF_OK or GF_NOT_CONVERGED (or the error)           */
  int32_t sweeps;          /* total overrelaxation sweeps (RED + BLACK = 1)      */
  int32_t sweeps_lo;       /* gf_fix_mixed: sweeps of the FP32 phase              */
  int32_t checks;          /* number of F/theta evaluations                       */
  double F, theta;         /* at the last check (Coulomb: mean F, max theta)      */
  double theta_at_switch;  /* gf_fix_mixed: theta when the FP32 phase ended        */
  double wall_ms;          /* host wall time of the call                          */
  /* GF_FLAG_TIMING: kernel time (ms) and launches: [0] FP32 sweeps, [1] FP64
   * sweeps, [2] measurement, [3] reunitarisation and conversion, [4]
   * annealing (heatbath and microcanonical half-sweeps), [5] reserved */
  double kernel_ms[6];
  int64_t kernel_launches[6];
  int32_t sa_steps;        /* annealing steps done                                 */
  int32_t frozen_slice_sweeps; /* GF_FLAG_FREEZE_TIMESLICES: sum over sweeps of the
                              number of frozen timeslices (work not done)         */
  int32_t check_log_n;     /* records written to params.check_log                  */
  double unitarity_max;    /* GF_FLAG_MONITOR: the largest unitarity deviation of
                              any check; else -1                                  */
} gf_fix_result;

/* Runs the annealing schedule of params (if sa_steps > 0), then sweeps U (in
 * geom's precision) with a check (reunitarise, F, theta) before the first
 * sweep and every check_every sweeps until theta < theta_target or
 * max_sweeps. Synchronises the context stream. */
gf_status gf_fix(gf_ctx* ctx, void* U, const gf_geom* geom, int32_t gauge,
                 const gf_fix_params* params, gf_fix_result* result);
/* Mixed precision. U_hi (FP64) holds the input and receives the result;
 * U_lo (FP32, same extents, must not overlap U_hi) is workspace. The input is
 * converted to FP32 and swept until theta < theta_switch while the
 * accumulated site transformations g(x) are tracked (FP32, held by the
 * context); then g is projected onto SU(3) in FP64 and applied to the FP64
 * input, U_hi <- g(x) U_hi g(x+mu)^dag, so the FP64 phase starts exactly on
 * the gauge orbit of the input, and U_hi is swept until theta <
 * theta_target. With GF_FLAG_NO_TRACK the FP32 field itself is converted back
 * (reunitarised in FP64) instead; its gauge-invariant content then carries
 * the FP32 rounding of the first phase. */
gf_status gf_fix_mixed(gf_ctx* ctx, void* U_lo, const gf_geom* geom_lo, void* U_hi,
                       const gf_geom* geom_hi, int32_t gauge, const gf_fix_params* params,
                       gf_fix_result* result);

/* ---- batches (Gribov copies, lattices of uneven extents) ------------------- */
/* n independent Landau problems fixed together: every annealing step,
 * half-sweep, reunitarisation and measurement is one launch over all lattices
 * that are still active (each lattice leaves a phase at its own check), and
 * the sweeps between checks are replayed from a hipGraph.
 * geoms: n FP64 geometries (extents may differ; all of one storage);
 * U: n caller-owned FP64 device fields, borrowed until gf_batch_destroy;
 * they hold the inputs and receive the results. The batch allocates its FP32
 * 12-real working fields and FP32 gauge-transformation fields (192 + 48 bytes
 * per site, padded sites included) at creation. Coulomb batches are GF_ERR_UNSUPPORTED.
 * Sweep variant: the context's (gf_set_sweep_variant, gf_autotune,
 * gf_batch_autotune); with none set, the built-in one for the total size of
 * the active lattices' fields of the phase's precision (see
 * gf_set_sweep_variant). */
typedef struct gf_batch gf_batch;
gf_status gf_batch_create(gf_ctx* ctx, int32_t n, const gf_geom* geoms, void* const* U,
                          int32_t gauge, gf_batch** out);
/* The gf_fix_mixed pipeline per lattice (annealing in FP32 with g tracked if
 * sa_steps > 0, FP32 overrelaxation to theta_switch, FP64 transformation of
 * the input by g, FP64 overrelaxation to theta_target). The annealing draws of
 * lattice l use the key seed + l, so lattice l ends exactly where gf_fix_mixed
 * on it alone with seed + l ends. results: n host structs (kernel timings
 * are reported in results[0]). Synchronises the context stream. */
gf_status gf_batch_run(gf_batch* batch, const gf_fix_params* params, gf_fix_result* results);
/* Tunes the batch's overrelaxation sweeps, both phases: [0] FP32 12-real with
 * g tracked (on the batch's working fields, as gf_batch_run starts them),
 * [1] FP64 in the caller's storage (on scratch copies: the caller's fields
 * are not modified). Every lanes x nontemporal variant runs a block of
 * RED/BLACK sweep pairs over all lattices, captured as a hipGraph; the nine
 * blocks are replayed in turn for five rounds and each variant timed by its
 * median. The fastest of each phase is kept on the context for the phase's
 * precision and storage and the size class of the batch's fields of that
 * precision (so it applies while the active lattices' fields stay in that
 * class) and returned in tps_out[2], nt_out[2] (NULL allowed); ms_out (NULL
 * or 18 floats, index 9 * phase + 3 * nontemporal + log2(tps)): the time per
 * half-sweep. Allocates the FP64 scratch copies (the fields' total size) for
 * the call; synchronises the context stream. */
gf_status gf_batch_autotune(gf_batch* batch, int32_t* tps_out, int32_t* nt_out, float* ms_out);
gf_status gf_batch_destroy(gf_batch* batch);

#ifdef __cplusplus
}
#endif
#endif /* GF_H */
