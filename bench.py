"""Benchmark: Landau overrelaxation gauge fixing on one MI355X.

Headline workload (default, --workload landau48): a 48^4 SU(3) configuration
from a quenched Wilson-action heatbath at beta = 6.2 (cold start, 400 sweeps,
Philox seed 3), generated on the GPU before anything is timed; the field
(2.04 GB in FP64 12-real storage) is eight times the 256 MB Infinity Cache,
so the sweeps run at HBM speed.

One benchmark step is a fixed block of that configuration's gauge fixing:
1000 sweeps (RED + BLACK half-sweeps, omega = 1.7) of the FP64 12-real field,
replayed from a captured hipGraph of 100 sweeps, with the F/theta check
(reunitarisation, F, theta in FP64) every 100 sweeps -- the FP64 phase that
takes most of the time of the mixed-precision fix. The steps continue one
fix of the input. value = site updates per second over the timed steps
(V x sweeps / time); the roofline object reports the FP64 12-real sweep
kernel (HIP events around its launches in the timed steps).

Beside the steps, run once each and timed in full: the mixed-precision fix
(FP32 12-real with g tracked until theta < 1e-6, FP64 projection and
transformation, FP64 12-real until theta < 1e-14) and the pure-FP64 fix of the
same input to theta < 1e-14, giving the mixed-vs-FP64 time to theta and the
final-F difference; the same pair on the 32^4 beta = 6.0 configuration
(300 sweeps, seed 2), whose FP64 field (403 MB) the Infinity Cache partly
holds; the storage variants; bandwidth probes; and the CPU oracle timed on a
bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
FLOP_PER_SITE = 2253  # paper's count per site update (751 per SU(2) subgroup)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=str, default="32,32,32,32")
    ap.add_argument("--beta", type=float, default=6.0)
    ap.add_argument("--therm", type=int, default=300)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--omega", type=float, default=1.7)
    ap.add_argument("--theta-switch", type=float, default=1e-6)
    ap.add_argument("--late-switch", type=float, default=1e-12,
                    help="landau48/landau32: one more full mixed fix that leaves FP32 at this "
                         "theta (0: skip)")
    ap.add_argument("--theta-target", type=float, default=1e-14)
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--max-sweeps", type=int, default=20000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64-only comparison and the variant table")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in sweep variants")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the sweeps between checks one by one instead of replaying a "
                         "captured hipGraph")
    ap.add_argument("--block", type=int, default=1000,
                    help="landau48: sweeps per benchmark step")
    ap.add_argument("--workload", default="landau48",
                    choices=("landau48", "landau32", "coulomb", "batch", "scan", "mag"),
                    help="landau48 (default, the benchmark line): 48^4 beta 6.2, steps are "
                         "1000-sweep blocks of the FP64 fix, plus the full mixed and FP64 fixes; "
                         "landau32: 32^4 beta 6.0, each step a full mixed fix; coulomb: 32^3x64 beta 6.0 with "
                         "3000 annealing steps then the mixed Coulomb fix; batch: 64 Haar copies "
                         "each of 16^4, 24^4, 12^3x24 with 2000 annealing steps then the mixed fix; "
                         "scan: 32^4 sweeps and time against the precision switch, omega and the "
                         "stochastic-relaxation probability; mag: 32^4 maximally Abelian gauge")
    ap.add_argument("--check-log", type=str, default="",
                    help="write the check logs of the full mixed and FP64 fixes (one JSON "
                         "line per check: sweeps, precision, F, theta, unitarity deviation, "
                         "elapsed ms) to this file")
    ap.add_argument("--variant", type=str, default="",
                    help="probe: lanes,nontemporal of the FP64 12-real sweep (the benchmark's "
                         "tuned variant), e.g. 4,2")
    ap.add_argument("--all-variants", action="store_true",
                    help="probe: also 2 sweeps of every lanes x nontemporal variant of the "
                         "12-real sweeps (counter runs then cover any tuned variant)")
    ap.add_argument("--probe", action="store_true",
                    help="kernel probe for profilers: bandwidth probes of known size, then "
                         "20 sweeps of each storage variant on a generated input")
    return ap.parse_args()


def stream_probes(ctx, torch, nbytes=2 * 1024 ** 3, reps=10):
    """Copy, in-place read-modify-write and read-only streams of known size."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    out = {}
    for kind, name, moved in ((0, "copy", 2), (1, "rmw", 2), (2, "read", 1)):
        ctx.stream_probe(a, b, nbytes, kind)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            ctx.stream_probe(a, b, nbytes, kind)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        out[name + "_GBps"] = round(reps * moved * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    return out


def variant_rates(ctx, torch, gf, canon, dims, omega, n=100):
    V = 1
    for d in dims:
        V *= d
    var = {}
    for prec, st in ((gf.FP32, gf.R12), (gf.FP32, gf.R18), (gf.FP64, gf.R12), (gf.FP64, gf.R18)):
        g = gf.Geom.make(dims, prec, st)
        f = ctx.empty_field(g)
        ctx.pack(g, canon, f)
        for _ in range(4):
            ctx.sweep(f, g, gf.LANDAU, 0, omega)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for k in range(n):
            ctx.sweep(f, g, gf.LANDAU, 0, omega)
            ctx.sweep(f, g, gf.LANDAU, 1, omega)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        sups = V * n / (ms * 1e-3)
        gbs = sups * 16 * st * prec / 1e9
        name = ("fp32" if prec == gf.FP32 else "fp64") + ("_r12" if st == gf.R12 else "_r18")
        var[name] = {"site_updates_per_s": round(sups, 0),
                     "gflops": round(sups * FLOP_PER_SITE / 1e9, 1),
                     "GBps": round(gbs, 1), "frac_peak": round(gbs / PEAK_HBM_GBS, 4),
                     "us_per_half_sweep": round(1e3 * ms / (2 * n), 2),
                     "variant": dict(zip(("lanes_per_site", "nontemporal"),
                                         ctx.sweep_variant_for(g)))}
        del f
    return var


def hbm_traffic(kname, dims):
    """HBM bytes per launch of kname from the committed counter summary, or None
    when there is none for this lattice or the kernel sources changed since."""
    import prof_summary

    path = os.path.join(ROOT, "profiles", "sweep_hbm_counters_%s.md" % "x".join(map(str, dims)))
    data = prof_summary.load_counters(path)
    if not data or data.get("kernel_source_hash") != prof_summary.kernel_source_hash():
        return None
    k = data["kernels"].get(kname)
    return round(k["traffic_bytes"]) if k else None


def coulomb_main(args):
    """32^3 x 64 Coulomb gauge: annealing (T 1.45 -> 0.01 over 3000 steps, 3
    microcanonical sweeps each) then FP32 -> FP64 overrelaxation to theta < 1e-14,
    twice from the same start: all 64 timeslices in every launch, then with
    each timeslice frozen once its theta_t is below the phase's target."""
    import torch

    import inputs
    import paper_1209_4008_amd as gf

    dims = (64, 32, 32, 32)
    V = 64 * 32 ** 3
    Vs = V // 64
    ctx = gf.Context(0)
    canon = inputs.gpu_heatbath(dims, 6.0, args.therm, 4, progress=100)
    glo = gf.Geom.make(dims, gf.FP32, gf.R12)
    ghi = gf.Geom.make(dims, gf.FP64, gf.R12)
    U_lo, U_hi = ctx.empty_field(glo), ctx.empty_field(ghi)
    for g, f in ((glo, U_lo), (ghi, U_hi)):
        ctx.pack(g, canon, f)
        ctx.autotune(g, gf.COULOMB, U_like=f)
    # the annealing updates run in FP32 with g tracked; tuned at a mid-schedule T
    ctx.pack(glo, canon, U_lo)
    anneal_tuned = ctx.autotune_anneal(glo, gf.COULOMB, U_like=U_lo, T=0.7)
    log("annealing variant", anneal_tuned)

    def run(extra_flags):
        ctx.pack(ghi, canon, U_hi)
        P0 = ctx.empty_out(1)
        ctx.plaquette(U_hi, ghi, P0)
        # a few timeslices pass near saddle points of F, where theta_t rises by
        # orders of magnitude before the sweeps reach a maximum; the fix ends
        # when the last timeslice is below the target, so the cap is generous
        p = gf.fix_params(omega=args.omega, theta_target=1e-14, theta_switch=1e-6,
                          max_sweeps=max(args.max_sweeps, 100000), check_every=args.check_every,
                          flags=gf.FLAG_TIMING | gf.FLAG_GRAPH | extra_flags, sa_steps=3000,
                          sa_micro=3, sa_T0=1.45, sa_T1=0.01, sa_reunit_every=10, seed=4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.fix_mixed(U_lo, glo, U_hi, ghi, gf.COULOMB, p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        F, th, P1 = ctx.empty_out(64), ctx.empty_out(64), ctx.empty_out(1)
        ctx.measure(U_hi, ghi, gf.COULOMB, F, th)
        ctx.plaquette(U_hi, ghi, P1)
        sa_ms, sa_n = r.kernel_ms[4], r.kernel_launches[4]
        or_ms = r.kernel_ms[0] + r.kernel_ms[1]
        updates = V * r.sweeps - Vs * r.frozen_slice_sweeps
        return {"total_ms": round(1e3 * dt, 1), "status": r.status,
                "annealing": {"steps": r.sa_steps, "ms": round(sa_ms, 1),
                              "half_sweeps_per_s": round(sa_n / (sa_ms * 1e-3), 1),
                              "site_updates_per_s": round(V / 2 * sa_n / (sa_ms * 1e-3), 0)},
                "overrelaxation": {"sweeps": r.sweeps, "sweeps_fp32": r.sweeps_lo,
                                   "frozen_timeslice_sweeps": r.frozen_slice_sweeps,
                                   "ms": round(or_ms, 1),
                                   "site_updates_per_s": round(updates / (or_ms * 1e-3), 0),
                                   # 3 x (44 + 19 + 8 x 84) flop per site update with
                                   # the spatial K (the paper's Landau count is 2253)
                                   "gflops_2205": round(2205 * updates / (or_ms * 1e-3) / 1e9, 1)},
                "theta_t_max": float(th.max().item()),
                "theta_t_median": float(th.median().item()),
                "timeslices_below_1e-14": int((th < 1e-14).sum().item()),
                "F_t_mean": float(F.mean().item()),
                "plaquette_change": abs(P1.item() - P0.item())}

    full = run(0)
    print("all timeslices:", json.dumps(full), file=sys.stderr, flush=True)
    frozen = run(gf.FLAG_FREEZE_TIMESLICES)
    out = {"metric": "Coulomb gauge fixing with annealing: time to max_t theta_t < 1e-14",
           "workload": "coulomb 32^3x64 beta=6.0, 3000 annealing steps (T 1.45->0.01, 3 micro), "
                       "mixed fp32-r12 -> fp64-r12 omega=%g" % args.omega,
           "all_timeslices": full, "freeze_converged_timeslices": frozen,
           "speedup_freeze": round(full["total_ms"] / frozen["total_ms"], 3)}
    ctx.close()
    print(json.dumps(out), flush=True)


def batch_main(args):
    """Gribov-copy batch: 64 Haar copies each of 16^4 (beta 5.8), 24^4 (6.0) and
    12^3 x 24 (5.9) heatbath configurations, annealing 2000 steps (T 1.2 -> 0.01,
    3 micro) then the mixed fix to theta < 1e-13, all in one batch; then the same
    copies with overrelaxation only, for the best-F comparison."""
    import numpy as np
    import torch

    import inputs
    import paper_1209_4008_amd as gf

    bases = [((16, 16, 16, 16), 5.8, 5), ((24, 24, 24, 24), 6.0, 6), ((24, 12, 12, 12), 5.9, 7)]
    copies = 64
    ctx = gf.Context(0)
    canon = []
    for dims, beta, seed in bases:
        canon.append(inputs.gpu_heatbath(dims, beta, args.therm, seed))
    torch.cuda.synchronize()
    geoms, fields, owner = [], [], []
    for k, (dims, beta, seed) in enumerate(bases):
        g = gf.Geom.make(dims, gf.FP64, gf.R12)
        for cp in range(copies):
            c = canon[k].clone()
            inputs.gpu_haar_copy(c, dims, 1000 + seed, cp)
            f = ctx.empty_field(g)
            ctx.pack(g, c, f)
            geoms.append(g)
            fields.append(f)
            owner.append(k)
    sites = sum(g.volume for g in geoms)
    pristine = [f.clone() for f in fields]
    out = {"metric": "Gribov-copy batch: copies/s and best F per base configuration",
           "workload": "64 Haar copies each of 16^4 b5.8, 24^4 b6.0, 12^3x24 b5.9; annealing "
                       "2000 steps (T 1.2->0.01, 3 micro) + mixed fix theta<1e-13, one batch",
           "lattices": len(geoms), "sites": sites}
    if not args.no_tune:
        # the batch tuner: both phases' sweeps over all 192 fields (5.4 GB FP32,
        # 10.8 GB FP64), kept on the context for their size class
        b = gf.Batch(ctx, geoms, fields)
        v32, v64, times = b.autotune()
        b.close()
        out["autotune"] = {
            ph: {"lanes_per_site": v[0], "nontemporal": v[1],
                 "us_per_half_sweep": {f"tps{k[1]}_nt{k[2]}": round(t * 1e3, 1)
                                       for k, t in times.items() if k[0] == i}}
            for i, (ph, v) in enumerate((("fp32_tracked", v32), ("fp64", v64)))}
        log("batch autotune", json.dumps(out["autotune"]))
    for label, sa in (("annealed", 2000), ("overrelaxation_only", 0)):
        for f, p0 in zip(fields, pristine):
            f.copy_(p0)
        b = gf.Batch(ctx, geoms, fields)
        p = gf.fix_params(omega=args.omega, theta_target=1e-13, theta_switch=1e-6,
                          max_sweeps=args.max_sweeps, check_every=args.check_every,
                          flags=gf.FLAG_TIMING | gf.FLAG_GRAPH, sa_steps=sa, sa_micro=3,
                          sa_T0=1.2, sa_T1=0.01, sa_reunit_every=10, seed=11)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = b.run(p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.close()
        Fs = np.array([r.F for r in res])
        per_base = {}
        for k, (dims, beta, seed) in enumerate(bases):
            sel = Fs[np.array(owner) == k]
            per_base["x".join(map(str, dims))] = {
                "best_F": float(sel.max()), "mean_F": float(sel.mean()),
                "min_F": float(sel.min()),
                "copies_within_1e-8_of_best": int((sel > sel.max() - 1e-8).sum())}
        out[label] = {"total_ms": round(1e3 * dt, 1), "copies_per_s": round(len(geoms) / dt, 2),
                      "converged": int(sum(r.status == gf.OK for r in res)),
                      "mean_sweeps": float(np.mean([r.sweeps for r in res])),
                      "annealing_ms": round(res[0].kernel_ms[4], 1),
                      "per_base": per_base}
        log(label, json.dumps(out[label]))
    ctx.close()
    print(json.dumps(out), flush=True)


def mag_main(args):
    """Maximally Abelian gauge on the 32^4 beta = 6.0 configuration: the mixed
    driver (FP32 12-real with g tracked to theta_MAG < 1e-8, FP64 12-real to
    theta_MAG < 1e-12) against pure FP64, with the per-half-sweep time of the
    MAG kernels and their algorithmic bandwidth."""
    import torch

    import inputs
    import paper_1209_4008_amd as gf

    dims = (32, 32, 32, 32)
    V = 32 ** 4
    ctx = gf.Context(0)
    canon = inputs.gpu_heatbath(dims, 6.0, 300, 2, progress=100)
    glo = gf.Geom.make(dims, gf.FP32, gf.R12)
    ghi = gf.Geom.make(dims, gf.FP64, gf.R12)
    U_lo, U_hi = ctx.empty_field(glo), ctx.empty_field(ghi)
    tuning = {}
    for g, f in ((glo, U_lo), (ghi, U_hi)):
        ctx.pack(g, canon, f)
        best, ms = ctx.autotune(g, gf.MAG, U_like=f)
        tuning["fp32" if g.prec == gf.FP32 else "fp64"] = {
            "lanes_per_site": best[0], "nontemporal": best[1],
            "us_per_half_sweep": {f"tps{k[0]}_nt{k[1]}": round(v * 1e3, 2) for k, v in ms.items()}}
    log("mag autotune", tuning)
    flags = gf.FLAG_TIMING | gf.FLAG_GRAPH
    p = gf.fix_params(omega=1.7, theta_target=1e-12, theta_switch=1e-8, max_sweeps=20000,
                      check_every=100, flags=flags)
    ctx.pack(ghi, canon, U_hi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.fix_mixed(U_lo, glo, U_hi, ghi, gf.MAG, p)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    ctx.pack(ghi, canon, U_hi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r64 = ctx.fix(U_hi, ghi, gf.MAG, p)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0

    def rate(ms, n, bytes_per_site):
        us = 1e3 * ms / max(n, 1)
        return {"us_per_half_sweep": round(us, 2),
                "GBps": round((V // 2) * bytes_per_site / (us * 1e-6) / 1e9, 1)}

    out = {"metric": "maximally Abelian gauge: time to theta_MAG < 1e-12, MAG sweep rates",
           "workload": "mag 32x32x32x32 wilson-heatbath beta=6 (300 sweeps, seed 2), omega 1.7, "
                       "mixed fp32-r12 (g tracked, to 1e-8) -> fp64-r12",
           "mixed": {"ms": round(1e3 * t_mixed, 1), "sweeps": r.sweeps, "sweeps_fp32": r.sweeps_lo,
                     "status": r.status, "F": r.F, "theta": r.theta,
                     "fp32_kernel": rate(r.kernel_ms[0], r.kernel_launches[0], 16 * 12 * 4 + 96),
                     "fp64_kernel": rate(r.kernel_ms[1], r.kernel_launches[1], 16 * 12 * 8)},
           "fp64_only": {"ms": round(1e3 * t64, 1), "sweeps": r64.sweeps, "status": r64.status,
                         "F": r64.F, "theta": r64.theta,
                         "fp64_kernel": rate(r64.kernel_ms[1], r64.kernel_launches[1],
                                             16 * 12 * 8)},
           "mixed_speedup_vs_fp64": round(t64 / t_mixed, 3),
           "F_rel_diff": abs(r.F - r64.F) / abs(r64.F),
           "site_updates_per_s_mixed": round(V * r.sweeps / t_mixed, 0),
           "autotune": tuning}
    ctx.close()
    print(json.dumps(out), flush=True)


def scan_main(args):
    """Tuning scans on 32^4 heatbath configurations (mixed FP32 -> FP64 driver,
    12-real storage, g tracked):
    (1) precision switch: the benchmark configuration (beta 6.0, seed 2) fixed
        to theta < 1e-14 with the FP32 -> FP64 switch at theta 1e-6 ... 1e-12,
        against pure FP64;
    (2) sweeps to theta < 1e-12 on three beta = 6.1 configurations (300 heatbath
        sweeps, seeds 8, 9, 10) against the overrelaxation parameter omega and against
        the stochastic-relaxation probability (omega = 1), the quantity the
        paper tunes for its beta = 6.1 32^4 lattice (Sec. 5, Fig. 2 left);
    (3) the same for the four forms of g^omega at omega 1.7 and 1.85, with
        the cost per half-sweep of each."""
    import torch

    import inputs
    import paper_1209_4008_amd as gf

    dims = (32, 32, 32, 32)
    cap = 30000
    ctx = gf.Context(0)
    glo = gf.Geom.make(dims, gf.FP32, gf.R12)
    ghi = gf.Geom.make(dims, gf.FP64, gf.R12)
    U_lo, U_hi = ctx.empty_field(glo), ctx.empty_field(ghi)
    out = {"metric": "sweeps and time to theta against the precision switch, omega and the "
                     "stochastic-relaxation probability",
           "workload": "32^4 wilson-heatbath beta 6.0 (seed 2) and beta 6.1 (seeds 8, 9, 10), "
                       "300 sweeps each; mixed fp32-r12 -> fp64-r12, check every 100 sweeps, "
                       "at most %d sweeps per precision phase" % cap}

    def run(canon, **kw):
        ctx.pack(ghi, canon, U_hi)
        prm = gf.fix_params(check_every=100, max_sweeps=cap, flags=gf.FLAG_GRAPH, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.fix_mixed(U_lo, glo, U_hi, ghi, gf.LANDAU, prm)
        torch.cuda.synchronize()
        return r, 1e3 * (time.perf_counter() - t0)

    canon = inputs.gpu_heatbath(dims, 6.0, 300, 2, progress=100)
    for g, f in ((glo, U_lo), (ghi, U_hi)):
        ctx.pack(g, canon, f)
        ctx.autotune(g, gf.LANDAU, U_like=f)
    ctx.pack(ghi, canon, U_hi)
    ref = gf.fix_params(omega=1.7, theta_target=1e-14, max_sweeps=cap, flags=gf.FLAG_GRAPH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r64 = ctx.fix(U_hi, ghi, gf.LANDAU, ref)
    torch.cuda.synchronize()
    t64 = 1e3 * (time.perf_counter() - t0)
    out["fp64_only"] = {"ms": round(t64, 1), "sweeps": r64.sweeps, "F": r64.F,
                        "theta": r64.theta, "status": r64.status}
    log(f"fp64 only: {r64.sweeps} sweeps {t64:.0f} ms")
    rows = []
    for sw in (1e-6, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11, 1e-12):
        r, ms = run(canon, omega=1.7, theta_target=1e-14, theta_switch=sw)
        rows.append({"theta_switch": sw, "ms": round(ms, 1), "sweeps": r.sweeps,
                     "sweeps_fp32": r.sweeps_lo, "theta_at_switch": r.theta_at_switch,
                     "theta": r.theta, "status": r.status,
                     "F_rel_diff_vs_fp64": abs(r.F - r64.F) / abs(r64.F),
                     "speedup_vs_fp64": round(t64 / ms, 3)})
        log("switch", rows[-1])
    out["switch_scan"] = rows

    # omega and stochastic-relaxation scans on three beta = 6.1 configurations
    # (seeds 8, 9, 10): each setting ends at its own Gribov copy, so the sweep
    # count of one configuration is noisy; the mean over three is reported too
    seeds = (8, 9, 10)
    canons = [inputs.gpu_heatbath(dims, 6.1, 300, sd, progress=100) for sd in seeds]
    rows = []
    for w in (1.0, 1.3, 1.5, 1.6, 1.65, 1.7, 1.75, 1.8, 1.85, 1.9, 1.95):
        per = []
        for sd, cn in zip(seeds, canons):
            r, ms = run(cn, omega=w, theta_target=1e-12, theta_switch=1e-9)
            per.append({"seed": sd, "sweeps": r.sweeps, "sweeps_fp32": r.sweeps_lo,
                        "converged": r.status == gf.OK, "ms": round(ms, 1), "F": r.F})
        rows.append({"omega": w, "mean_sweeps": sum(x["sweeps"] for x in per) / len(per),
                     "mean_ms": round(sum(x["ms"] for x in per) / len(per), 1), "configs": per})
        log("omega", w, [x["sweeps"] for x in per])
    out["omega_scan"] = rows
    rows = []
    for prob in (0.5, 0.7, 0.8, 0.85, 0.9, 0.95):
        per = []
        for sd, cn in zip(seeds, canons):
            r, ms = run(cn, omega=1.0, theta_target=1e-12, theta_switch=1e-9, sr_prob=prob,
                        seed=sd)
            per.append({"seed": sd, "sweeps": r.sweeps, "sweeps_fp32": r.sweeps_lo,
                        "converged": r.status == gf.OK, "ms": round(ms, 1), "F": r.F})
        rows.append({"sr_prob": prob, "mean_sweeps": sum(x["sweeps"] for x in per) / len(per),
                     "mean_ms": round(sum(x["ms"] for x in per) / len(per), 1), "configs": per})
        log("sr", prob, [x["sweeps"] for x in per])
    out["sr_scan"] = rows
    # forms of g^omega (0: the 19-flop form; 1, 2: first and second order of the
    # binomial series; 3: exact power) at omega 1.7 and 1.85: sweeps and cost
    rows = []
    canon = canons[0]
    for w in (1.7, 1.85):
        for form in (0, 1, 2, 3):
            ctx.pack(ghi, canon, U_hi)
            prm = gf.fix_params(omega=w, theta_target=1e-12, theta_switch=1e-9, check_every=100,
                                max_sweeps=cap, or_form=form, flags=gf.FLAG_GRAPH | gf.FLAG_TIMING)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.fix_mixed(U_lo, glo, U_hi, ghi, gf.LANDAU, prm)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            rows.append({"omega": w, "form": form, "sweeps": r.sweeps, "sweeps_fp32": r.sweeps_lo,
                         "converged": r.status == gf.OK, "ms": round(ms, 1), "F": r.F,
                         "us_per_half_sweep_fp32": round(1e3 * r.kernel_ms[0]
                                                         / max(r.kernel_launches[0], 1), 2),
                         "us_per_half_sweep_fp64": round(1e3 * r.kernel_ms[1]
                                                         / max(r.kernel_launches[1], 1), 2)})
            log("form", rows[-1])
    out["form_scan"] = rows
    ctx.close()
    print(json.dumps(out), flush=True)


def probe_main(args):
    """Short fixed workload for rocprofv3 runs (kernel trace or counters)."""
    import torch

    import inputs
    import paper_1209_4008_amd as gf

    dims = tuple(int(v) for v in args.dims.split(","))
    ctx = gf.Context(0)
    log("probe: stream probes (2 GiB, 10 reps each)")
    res = {"probe": stream_probes(ctx, torch)}
    canon = inputs.gpu_config0(dims, 0.3, args.seed)
    torch.cuda.synchronize()
    if not args.no_tune:
        for prec, st in ((gf.FP32, gf.R12), (gf.FP32, gf.R18), (gf.FP64, gf.R12), (gf.FP64, gf.R18)):
            g = gf.Geom.make(dims, prec, st)
            f = ctx.empty_field(g)
            ctx.pack(g, canon, f)
            ctx.autotune(g, gf.LANDAU, U_like=f)
            del f
    if args.variant:
        tps, nt = (int(v) for v in args.variant.split(","))
        ctx.set_sweep_variant(gf.FP64, gf.R12, tps, nt)
    log("probe: 20 sweeps per storage variant on", dims)
    res["variants"] = variant_rates(ctx, torch, gf, canon, dims, args.omega, n=20)
    if args.all_variants:
        # two sweeps of every lanes x nontemporal variant of the 12-real sweeps,
        # so that counter runs cover whichever variant a tuner picks
        log("probe: 2 sweeps of each 12-real variant")
        for prec in (gf.FP32, gf.FP64):
            g = gf.Geom.make(dims, prec, gf.R12)
            f = ctx.empty_field(g)
            ctx.pack(g, canon, f)
            for tps in (1, 2, 4):
                for nt in (0, 1, 2):
                    ctx.set_sweep_variant(prec, gf.R12, tps, nt)
                    for _ in range(2):
                        ctx.sweep(f, g, gf.LANDAU, 0, args.omega)
                        ctx.sweep(f, g, gf.LANDAU, 1, args.omega)
            ctx.set_sweep_variant(prec, gf.R12, 0, -1)
            torch.cuda.synchronize()
            del f
    ctx.close()
    print(json.dumps(res), flush=True)


def probe_batch_main(args):
    """Short batch run for rocprofv3 counter runs: the stream probes, then the
    192 lattices of the Gribov-copy batch (64 each of 16^4, 24^4, 12^3 x 24;
    random fields, which move the same bytes as heatbath ones) through 2
    annealing steps and 20 FP32 and 20 FP64 overrelaxation sweeps, every
    lattice active in every launch."""
    import torch

    import inputs
    import paper_1209_4008_amd as gf

    ctx = gf.Context(0)
    log("probe: stream probes (2 GiB, 10 reps each)")
    res = {"probe": stream_probes(ctx, torch)}
    geoms, fields = [], []
    for k, dims in enumerate(((16, 16, 16, 16), (24, 24, 24, 24), (24, 12, 12, 12))):
        g = gf.Geom.make(dims, gf.FP64, gf.R12)
        for cp in range(64):
            canon = inputs.gpu_config0(dims, 0.3, 100 * k + cp)
            f = ctx.empty_field(g)
            ctx.pack(g, canon, f)
            geoms.append(g)
            fields.append(f)
    torch.cuda.synchronize()
    sites = sum(g.volume for g in geoms)
    log("probe: batch of", len(geoms), "lattices,", sites, "sites")
    b = gf.Batch(ctx, geoms, fields)
    p = gf.fix_params(omega=args.omega, theta_target=1e-300, theta_switch=1e-300, max_sweeps=20,
                      check_every=10, sa_steps=2, sa_micro=1, sa_T0=1.0, sa_T1=0.5, seed=11)
    r = b.run(p)
    torch.cuda.synchronize()
    b.close()
    res["batch"] = {"lattices": len(geoms), "sites": sites, "sweeps": r[0].sweeps}
    ctx.close()
    print(json.dumps(res), flush=True)


def timed_fix(ctx, torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


def kernel_roofline(kms, kn, V, bytes_per_site, kname, dims):
    """achieved algorithmic bandwidth of a sweep kernel from pooled HIP-event
    timings (total ms, launches)"""
    per_launch = (V // 2) * bytes_per_site
    avg_ms = kms / max(kn, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": hbm_traffic(kname, dims),
            "kernel": kname, "avg_launch_us": round(avg_ms * 1e3, 3), "launches": kn,
            "bytes_per_launch": per_launch}


def tune_phases(ctx, gf, canon, pairs, gauge):
    tuning = {}
    for g, f in pairs:
        ctx.pack(g, canon, f)
        best, ms = ctx.autotune(g, gauge, U_like=f)
        name = ("fp32" if g.prec == gf.FP32 else "fp64") + ("_r12" if g.storage == gf.R12 else "_r18")
        tuning[name] = {"lanes_per_site": best[0], "nontemporal": best[1],
                        "us_per_half_sweep": {f"tps{k[0]}_nt{k[1]}": round(v * 1e3, 2)
                                              for k, v in ms.items()}}
        log(f"autotune {name}: {tuning[name]}")
    return tuning


def monitored(gf, params, n):
    """a copy of params with the unitarity monitor on and a check log of n records"""
    import ctypes as C
    p = type(params).from_buffer_copy(params)
    log_ = gf.check_log(n)
    p.flags |= gf.FLAG_MONITOR
    p.check_log = C.cast(log_, C.POINTER(gf.CheckRecord))
    p.check_log_cap = n
    return p, log_


def log_summary(gf, r, log_):
    """records of a fix's check log, and the largest unitarity deviation met at
    the checks of each precision"""
    recs = [log_[k].as_dict() for k in range(r.check_log_n)]
    worst = {}
    for e in recs:
        worst[e["precision"]] = max(worst.get(e["precision"], 0.0), e["unitarity"])
    return recs, {"checks_logged": len(recs),
                  "unitarity_max_at_checks": {k: float("%.3g" % v) for k, v in worst.items()}}


def mixed_vs_fp64(ctx, torch, gf, canon, glo, ghi, U_lo, U_hi, params, V, log_path=None):
    """the full mixed fix and the full FP64 fix of the same input, each timed,
    with the unitarity monitor and a check log (written as JSON lines to
    log_path if given)"""
    cap = params.max_sweeps * 2 // params.check_every + 8
    pm, log_m = monitored(gf, params, cap)
    ctx.pack(ghi, canon, U_hi)
    r, t_mixed = timed_fix(ctx, torch, lambda: ctx.fix_mixed(U_lo, glo, U_hi, ghi, gf.LANDAU, pm))
    log(f"mixed: {r.sweeps} sweeps ({r.sweeps_lo} FP32) in {t_mixed:.2f} s, theta {r.theta:.3e}")
    p64, log_64 = monitored(gf, params, cap)
    ctx.pack(ghi, canon, U_hi)
    r64, t64 = timed_fix(ctx, torch, lambda: ctx.fix(U_hi, ghi, gf.LANDAU, p64))
    log(f"fp64: {r64.sweeps} sweeps in {t64:.2f} s, theta {r64.theta:.3e}")
    recs_m, sum_m = log_summary(gf, r, log_m)
    recs_64, sum_64 = log_summary(gf, r64, log_64)
    if log_path:
        with open(log_path, "a") as fh:
            for run, recs in (("mixed", recs_m), ("fp64", recs_64)):
                for e in recs:
                    fh.write(json.dumps(dict(run=run, lattice=list(ghi.dims), **e)) + "\n")
    return r, t_mixed, r64, t64, {
        "mixed": {"time_ms": round(1e3 * t_mixed, 1), "sweeps": r.sweeps,
                  "sweeps_fp32": r.sweeps_lo, "status": r.status, "F": r.F, "theta": r.theta,
                  "site_updates_per_s": round(V * r.sweeps / t_mixed, 0), **sum_m},
        "fp64_only": {"time_ms": round(1e3 * t64, 1), "sweeps": r64.sweeps, "status": r64.status,
                      "F": r64.F, "theta": r64.theta,
                      "site_updates_per_s": round(V * r64.sweeps / t64, 0), **sum_64},
        "mixed_speedup_vs_fp64": round(t64 / t_mixed, 4),
        "final_F_rel_diff_mixed_vs_fp64": abs(r.F - r64.F) / abs(r64.F)}


def late_switch(ctx, torch, gf, canon, glo, ghi, U_lo, U_hi, params, switch, r64, t64):
    """the full mixed fix of the same input with the FP32 phase run on to theta
    < switch: time, sweeps and final F against the FP64 fix (r64, t64)"""
    p = type(params).from_buffer_copy(params)
    p.theta_switch = switch
    ctx.pack(ghi, canon, U_hi)
    r, t = timed_fix(ctx, torch, lambda: ctx.fix_mixed(U_lo, glo, U_hi, ghi, gf.LANDAU, p))
    log(f"mixed, switch {switch:g}: {r.sweeps} sweeps ({r.sweeps_lo} FP32) in {t:.2f} s, "
        f"theta {r.theta:.3e}")
    return {"theta_switch": switch, "time_ms": round(1e3 * t, 1), "sweeps": r.sweeps,
            "sweeps_fp32": r.sweeps_lo, "theta_at_switch": r.theta_at_switch,
            "status": r.status, "F": r.F, "theta": r.theta,
            "F_rel_diff_vs_fp64": abs(r.F - r64.F) / abs(r64.F),
            "speedup_vs_fp64": round(t64 / t, 4)}


def landau32_secondary(ctx, torch, gf, inputs, args):
    """32^4 beta 6.0 (300 sweeps, seed 2): mixed and FP64 fixes to theta < 1e-14
    and the FP64 sweep kernel's rate, which the Infinity Cache assists here."""
    dims = (32, 32, 32, 32)
    V = 32 ** 4
    canon = inputs.gpu_heatbath(dims, 6.0, 300, 2, progress=100)
    glo = gf.Geom.make(dims, gf.FP32, gf.R12)
    ghi = gf.Geom.make(dims, gf.FP64, gf.R12)
    U_lo, U_hi = ctx.empty_field(glo), ctx.empty_field(ghi)
    tuning = tune_phases(ctx, gf, canon, ((glo, U_lo), (ghi, U_hi)), gf.LANDAU)
    params = gf.fix_params(omega=args.omega, theta_target=1e-14, theta_switch=1e-6,
                           max_sweeps=args.max_sweeps, check_every=args.check_every,
                           flags=gf.FLAG_TIMING | gf.FLAG_GRAPH)
    r, t_mixed, r64, t64, out = mixed_vs_fp64(ctx, torch, gf, canon, glo, ghi, U_lo, U_hi,
                                              params, V, log_path=args.check_log or None)
    if args.late_switch > 0:
        out["mixed_late_switch"] = late_switch(ctx, torch, gf, canon, glo, ghi, U_lo, U_hi, params,
                                               args.late_switch, r64, t64)
    tps, nt = ctx.sweep_variant_for(ghi)
    kname = "k_update_half<double,6,0,UpdOR,%d,%d,false>" % (tps, nt)
    roof = kernel_roofline(r64.kernel_ms[1], r64.kernel_launches[1], V, 16 * 12 * 8, kname, dims)
    roof["infinity_cache_assisted"] = True
    out.update({"lattice": list(dims), "beta": 6.0, "roofline_fp64_sweep": roof,
                "autotune": tuning})
    del U_lo, U_hi, canon
    return out


def headline_main(args):
    import numpy as np
    import torch

    import inputs
    import paper_1209_4008_amd as gf

    dims = (48, 48, 48, 48)
    beta, therm, seed = 6.2, 400, 3
    V = int(np.prod(dims))
    torch.cuda.set_device(0)
    ctx = gf.Context(0)
    log("device", torch.cuda.get_device_name(0), "lattice", dims)
    t0 = time.time()
    canon = inputs.gpu_heatbath(dims, beta, therm, seed, progress=100)
    torch.cuda.synchronize()
    log(f"heatbath input ready in {time.time() - t0:.1f} s")
    g64c = gf.Geom.make(dims, gf.FP64, gf.R18)
    P = ctx.empty_out(1)
    tmp = ctx.empty_field(g64c)
    ctx.pack(g64c, canon, tmp)
    ctx.plaquette(tmp, g64c, P)
    plaq = P.item()
    del tmp
    log(f"plaquette {plaq:.6f}")
    glo = gf.Geom.make(dims, gf.FP32, gf.R12)
    ghi = gf.Geom.make(dims, gf.FP64, gf.R12)
    U_lo, U_hi = ctx.empty_field(glo), ctx.empty_field(ghi)
    axis = {}
    if not args.no_tune:
        # the storage axis: each storage's best variant, then the faster storage
        # (the benchmark runs 12 reals, the configuration's storage, either way);
        # the variants of the 12-real phases are then tuned once more, as the
        # benchmark runs them
        for g in (glo, ghi):
            best, ms = ctx.autotune_storage(g, gf.LANDAU, canon)
            axis["fp32" if g.prec == gf.FP32 else "fp64"] = {
                "fastest": "r12" if best == gf.R12 else "r18",
                "us_per_half_sweep": {"r12": round(ms[gf.R12] * 1e3, 2),
                                      "r18": round(ms[gf.R18] * 1e3, 2)}}
        log("autotune storage axis", axis)
    tuning = {} if args.no_tune else tune_phases(ctx, gf, canon, ((glo, U_lo), (ghi, U_hi)),
                                                 gf.LANDAU)
    if axis:
        tuning["storage_axis"] = axis
    flags = gf.FLAG_TIMING | (0 if args.no_graph else gf.FLAG_GRAPH)
    # a step: args.block sweeps of the FP64 fix of the input (theta_target 0:
    # the block always runs in full), checks every check_every sweeps
    block = gf.fix_params(omega=args.omega, theta_target=0.0, max_sweeps=args.block,
                          check_every=args.check_every, flags=flags)
    ctx.pack(ghi, canon, U_hi)
    for k in range(args.warmup):
        r = ctx.fix(U_hi, ghi, gf.LANDAU, block)
        log(f"warmup {k}: {r.sweeps} sweeps, theta {r.theta:.3e}, wall {r.wall_ms:.1f} ms")
    torch.cuda.synchronize()
    results = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        results.append(ctx.fix(U_hi, ghi, gf.LANDAU, block))
        log(f"step {k}: {results[-1].sweeps} sweeps, theta {results[-1].theta:.3e}, "
            f"F {results[-1].F:.12f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    sweeps = sum(r.sweeps for r in results)
    value = V * sweeps / elapsed
    tps, nt = ctx.sweep_variant_for(ghi)
    kname = "k_update_half<double,6,0,UpdOR,%d,%d,false>" % (tps, nt)
    roofline = kernel_roofline(sum(r.kernel_ms[1] for r in results),
                               sum(r.kernel_launches[1] for r in results), V, 16 * 12 * 8,
                               kname, dims)
    log("roofline", roofline)

    full_params = gf.fix_params(omega=args.omega, theta_target=args.theta_target,
                                theta_switch=args.theta_switch,
                                max_sweeps=max(args.max_sweeps, 60000),
                                check_every=args.check_every, flags=flags)
    extras = {}
    r, t_mixed, r64, t64, cmp = mixed_vs_fp64(ctx, torch, gf, canon, glo, ghi, U_lo, U_hi,
                                              full_params, V, log_path=args.check_log or None)
    extras.update(cmp)
    extras["mixed_fp64_phase_roofline"] = kernel_roofline(r.kernel_ms[1], r.kernel_launches[1],
                                                          V, 16 * 12 * 8, kname, dims)
    if args.late_switch > 0:
        extras["mixed_late_switch"] = late_switch(ctx, torch, gf, canon, glo, ghi, U_lo, U_hi,
                                                  full_params, args.late_switch, r64, t64)
    del U_lo, U_hi
    if not args.no_extras:
        extras["variants"] = variant_rates(ctx, torch, gf, canon, dims, args.omega, n=50)
        extras.update(stream_probes(ctx, torch))
        for probe in ("copy", "rmw"):
            key = probe + "_GBps"
            if extras.get(key):
                roofline["frac_of_measured_" + probe] = round(roofline["achieved"] / extras[key], 4)
        extras["landau32"] = landau32_secondary(ctx, torch, gf, inputs, args)
        l32 = extras["landau32"]["roofline_fp64_sweep"]
        if extras.get("copy_GBps"):
            l32["frac_of_measured_copy"] = round(l32["achieved"] / extras["copy_GBps"], 4)
    extras["autotune"] = tuning

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(canon, dims, args)
        if not args.no_extras:
            extras.update(cpu_extras(canon, dims, args, ctx, torch, gf, sweeps_1t=1))
        if cpu and cpu.get("value"):
            n = r64.sweeps
            extras["oracle_fp64_time_to_theta_extrapolated"] = {
                "s": round(V * n / cpu["value"], 1), "sweeps": n,
                "basis": "FP64 sweeps of the GPU's pure-FP64 run x V / the oracle's "
                         "site-updates/s on %d host threads (extrapolated, not run)" % cpu["cores"]}
    out = {
        "metric": "Landau OR site-updates/s, HBM GB/s %peak; mixed vs FP64 time-to-theta<1e-14",
        "value": round(value, 1),
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "landau-gauge-fix 48x48x48x48 wilson-heatbath beta=6.2 (400 sweeps, "
                               "seed 3): each step %d sweeps of the fp64-r12 fix (omega %g, check "
                               "every %d, hipGraph); beside it the full mixed fp32-r12 -> fp64-r12 "
                               "(switch %g) and pure fp64-r12 fixes to theta<%g, and the mixed "
                               "fix with the switch at %g"
                               % (args.block, args.omega, args.check_every, args.theta_switch,
                                  args.theta_target, args.late_switch),
                   "lattice": list(dims), "beta": beta, "omega": args.omega,
                   "check_every": args.check_every, "plaquette": round(plaq, 6),
                   "sweeps_per_step": sweeps / args.steps,
                   "gflops_2253": round(value * FLOP_PER_SITE / 1e9, 1)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.probe:
        if args.workload == "batch":
            probe_batch_main(args)
        else:
            probe_main(args)
        return
    if args.workload == "coulomb":
        coulomb_main(args)
        return
    if args.workload == "batch":
        batch_main(args)
        return
    if args.workload == "scan":
        scan_main(args)
        return
    if args.workload == "mag":
        mag_main(args)
        return
    if args.workload == "landau48":
        headline_main(args)
        return
    import numpy as np
    import torch

    import inputs
    import paper_1209_4008_amd as gf

    dims = tuple(int(v) for v in args.dims.split(","))
    V = int(np.prod(dims))
    torch.cuda.set_device(0)
    ctx = gf.Context(0)
    stream = ctx.stream
    log("device", torch.cuda.get_device_name(0), "lattice", dims)

    # ---- input: heatbath configuration generated on the GPU (not timed) ----
    t0 = time.time()
    canon = inputs.gpu_heatbath(dims, args.beta, args.therm, args.seed, progress=100)
    torch.cuda.synchronize()
    log(f"heatbath input ready in {time.time() - t0:.1f} s")
    g64c = gf.Geom.make(dims, gf.FP64, gf.R18)
    P = ctx.empty_out(1)
    tmp = ctx.empty_field(g64c)
    ctx.pack(g64c, canon, tmp)
    ctx.plaquette(tmp, g64c, P)
    plaq = P.item()
    del tmp
    log(f"plaquette {plaq:.6f}")

    glo = gf.Geom.make(dims, gf.FP32, gf.R12)
    ghi = gf.Geom.make(dims, gf.FP64, gf.R12)
    U_lo = ctx.empty_field(glo)
    U_hi = ctx.empty_field(ghi)
    tuning = {}
    if not args.no_tune:
        for g, f in ((glo, U_lo), (ghi, U_hi)):
            ctx.pack(g, canon, f)
            best, ms = ctx.autotune(g, gf.LANDAU, U_like=f)
            name = ("fp32" if g.prec == gf.FP32 else "fp64") + "_r12"
            tuning[name] = {"lanes_per_site": best[0], "nontemporal": best[1],
                            "us_per_half_sweep": {f"tps{k[0]}_nt{k[1]}": round(v * 1e3, 2)
                                                  for k, v in ms.items()}}
            log(f"autotune {name}: {tuning[name]}")
    flags = gf.FLAG_TIMING | (0 if args.no_graph else gf.FLAG_GRAPH)
    params = gf.fix_params(omega=args.omega, theta_target=args.theta_target,
                           theta_switch=args.theta_switch, max_sweeps=args.max_sweeps,
                           check_every=args.check_every, flags=flags)

    def step():
        ctx.pack(ghi, canon, U_hi)
        return ctx.fix_mixed(U_lo, glo, U_hi, ghi, gf.LANDAU, params)

    for k in range(args.warmup):
        r = step()
        log(f"warmup {k}: sweeps {r.sweeps} (fp32 {r.sweeps_lo}) theta {r.theta:.3e} "
            f"wall {r.wall_ms:.1f} ms")
    torch.cuda.synchronize()
    results = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        results.append(step())
        log(f"step {k}: sweeps {results[-1].sweeps} (fp32 {results[-1].sweeps_lo}) "
            f"theta {results[-1].theta:.3e} F {results[-1].F:.12f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    sweeps = sum(r.sweeps for r in results)
    value = V * sweeps / elapsed

    # ---- dominant kernel: HIP-event timings of the sweep launches in the timed steps ----
    kms = [sum(r.kernel_ms[i] for r in results) for i in range(4)]
    kn = [sum(r.kernel_launches[i] for r in results) for i in range(4)]
    # FP32 R12 sweep with the gauge transformation tracked (+2 x 12 reals), FP64 R12 sweep
    bytes_per_site = {0: 16 * 12 * 4 + 2 * 12 * 4, 1: 16 * 12 * 8}
    dom = 0 if kms[0] >= kms[1] else 1
    per_launch_bytes = (V // 2) * bytes_per_site[dom]
    avg_ms = kms[dom] / max(kn[dom], 1)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    tps, nt = ctx.sweep_variant_for(glo if dom == 0 else ghi)
    kname = "k_update_half<%s,6,0,UpdOR,%d,%d,%s>" % (
        "float" if dom == 0 else "double", tps, nt, "true" if dom == 0 else "false")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": hbm_traffic(kname, dims),
                "kernel": kname, "avg_launch_us": round(avg_ms * 1e3, 3), "launches": kn[dom],
                "bytes_per_launch": per_launch_bytes}

    extras = {}
    if not args.no_extras:
        # pure FP64 (12 reals) on the same input, same cadence
        gsave = ctx.empty_field(ghi)
        ctx.pack(ghi, canon, gsave)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r64 = ctx.fix(gsave, ghi, gf.LANDAU, params)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        mixed = results[-1]
        extras["fp64_only"] = {"time_ms": round(1e3 * t64, 2), "sweeps": r64.sweeps,
                               "F": r64.F, "theta": r64.theta}
        extras["mixed"] = {"time_ms": round(ms_per_step, 2), "sweeps": mixed.sweeps,
                           "sweeps_fp32": mixed.sweeps_lo, "F": mixed.F, "theta": mixed.theta}
        extras["mixed_speedup_vs_fp64"] = round(t64 / (ms_per_step * 1e-3), 4)
        extras["final_F_rel_diff_mixed_vs_fp64"] = abs(mixed.F - r64.F) / abs(r64.F)
        del gsave
        extras["variants"] = variant_rates(ctx, torch, gf, canon, dims, args.omega)
        extras.update(stream_probes(ctx, torch))
        # the same achieved rate against what plain streaming kernels reach on
        # this GPU (copy: read + write of 2 GiB; rmw: in-place read-modify-write)
        for probe in ("copy", "rmw"):
            key = probe + "_GBps"
            if extras.get(key):
                roofline["frac_of_measured_" + probe] = round(achieved / extras[key], 4)
    extras["autotune"] = tuning

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(canon, dims, args)
        if not args.no_extras:
            extras.update(cpu_extras(canon, dims, args, ctx, torch, gf))
            if "fp64_only" in extras and cpu and cpu.get("value"):
                # a full FP64 oracle fix of this input would take too long to
                # run; its time follows from the GPU run's sweep count (the same
                # sequence of sweeps) and the oracle's measured rate
                n = extras["fp64_only"]["sweeps"]
                extras["oracle_fp64_time_to_theta_extrapolated"] = {
                    "s": round(V * n / cpu["value"], 1), "sweeps": n,
                    "basis": "FP64 sweeps of the GPU's pure-FP64 run x V / the oracle's "
                             "site-updates/s on %d host threads (extrapolated, not run)" % cpu["cores"]}

    out = {
        "metric": "Landau OR site-updates/s, HBM GB/s %peak; mixed vs FP64 time-to-theta<1e-14",
        "value": round(value, 1),
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": "landau-gauge-fix %dx%dx%dx%d wilson-heatbath beta=%g (%d sweeps, seed %d), "
                               "mixed fp32-r12 -> fp64-r12, omega=%g, theta<%g (switch %g)"
                               % (dims + (args.beta, args.therm, args.seed, args.omega,
                                          args.theta_target, args.theta_switch)),
                   "lattice": list(dims), "beta": args.beta, "omega": args.omega,
                   "check_every": args.check_every, "plaquette": round(plaq, 6),
                   "sweeps_per_step": sweeps / args.steps,
                   "gflops_2253": round(value * FLOP_PER_SITE / 1e9, 1)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    ctx.close()
    print(json.dumps(out), flush=True)


def cpu_baseline(canon, dims, args):
    """The FP64 oracle, untuned, on the host cores: overrelaxation sweeps of the
    same configuration, as many as fit in about args.cpu_seconds."""
    import numpy as np

    import oracle

    U = canon.cpu().numpy().view(np.complex128).reshape(tuple(dims) + (4, 3, 3)).copy()
    V = int(np.prod(dims))
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    oracle.sweep(U, oracle.LANDAU, 0, args.omega)
    oracle.sweep(U, oracle.LANDAU, 1, args.omega)
    one = time.perf_counter() - t0
    n = max(1, int(args.cpu_seconds / max(one, 1e-6)) - 1)
    t0 = time.perf_counter()
    for _ in range(n):
        oracle.sweep(U, oracle.LANDAU, 0, args.omega)
        oracle.sweep(U, oracle.LANDAU, 1, args.omega)
    dt = time.perf_counter() - t0
    log(f"cpu oracle: {n} sweeps in {dt:.1f} s on {threads} threads")
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(V * n / dt, 1), "unit": "site-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} FP64 overrelaxation sweeps (omega {args.omega}) of the "
                      f"{'x'.join(map(str, dims))} input, canonical 18-real layout",
            "host": {"cpu_model": model, "nproc": os.cpu_count(),
                     "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}}


def cpu_extras(canon, dims, args, ctx, torch, gf, sweeps_1t=2):
    """The oracle on one host thread (2 sweeps of the same input), and the
    8^4 configuration 0 fixed to theta < 1e-12 in FP64 by the oracle (all host
    threads) and by the GPU (12 reals, same cadence)."""
    import numpy as np

    import inputs
    import oracle

    out = {}
    U = canon.cpu().numpy().view(np.complex128).reshape(tuple(dims) + (4, 3, 3)).copy()
    V = int(np.prod(dims))
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        for _ in range(sweeps_1t):
            oracle.sweep(U, oracle.LANDAU, 0, args.omega)
            oracle.sweep(U, oracle.LANDAU, 1, args.omega)
        dt = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    out["cpu_oracle_1_thread"] = {"site_updates_per_s": round(sweeps_1t * V / dt, 1),
                                  "sample": "%d FP64 sweeps of the benchmark input" % sweeps_1t}
    d0 = (8, 8, 8, 8)
    U0 = inputs.config0(d0, 0.3, 1)
    ref = U0.copy()
    ref[..., 2, :] = np.conj(np.cross(ref[..., 0, :], ref[..., 1, :]))  # the 12-real input
    t0 = time.perf_counter()
    ro = oracle.fix(ref, oracle.LANDAU, args.omega, 1e-12, 2000, 100, 1)
    t_cpu = time.perf_counter() - t0
    g0 = gf.Geom.make(d0, gf.FP64, gf.R12)
    f0 = ctx.empty_field(g0)
    c0 = torch.from_numpy(U0.view(np.float64).reshape(-1).copy()).to("cuda")
    p0 = gf.fix_params(omega=args.omega, theta_target=1e-12, max_sweeps=2000, check_every=100,
                       flags=gf.FLAG_GRAPH)
    ctx.pack(g0, c0, f0)
    ctx.fix(f0, g0, gf.LANDAU, p0)  # warm-up (graph capture, first launches)
    ctx.pack(g0, c0, f0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0 = ctx.fix(f0, g0, gf.LANDAU, p0)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    out["config0_8x8x8x8_time_to_theta_1e-12"] = {
        "oracle_ms": round(1e3 * t_cpu, 1), "oracle_threads": threads, "oracle_sweeps": ro["sweeps"],
        "gpu_ms": round(1e3 * t_gpu, 2), "gpu_sweeps": r0.sweeps,
        "F_rel_diff": abs(r0.F - ro["F"]) / abs(ro["F"])}
    log("cpu extras", out)
    return out


if __name__ == "__main__":
    main()
