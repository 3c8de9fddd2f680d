"""Summaries of rocprofv3 output for the profiles/ folder.

  python prof_summary.py kernels STATS_CSV --command CMD
  python prof_summary.py counters FETCH_CSV WRITE_CSV --command CMD
  python prof_summary.py busy TRACE_CSV --match REGEX --command CMD

Measurement support for bench.py and profiles/, not part of the library.
`kernels` turns a --kernel-trace --stats kernel_stats.csv into a table of
calls and average durations. `counters` turns two --pmc runs (FETCH_SIZE, then
WRITE_SIZE, in KiB per dispatch) of `bench.py --probe` into HBM bytes per
dispatch, each counter scaled by what it reads for the copy probe of known
size (2 GiB read + 2 GiB written per dispatch), and compares the sweep kernels
with their algorithmic bytes. Both embed the hash of the kernel sources so that
a reader (bench.py) can tell whether the kernels changed since. `busy` splits a
--kernel-trace kernel_trace.csv into stretches of GPU work separated by idle
gaps longer than --split-ms (host-side set-up between runs) and reports, for
each stretch that holds a kernel matching REGEX, how much of its wall time had
a kernel running: the idle share a driver's host-side checks and launches cost.
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("paper_1209_4008_amd/csrc/gf_device.hpp", "paper_1209_4008_amd/csrc/gf_kernels.hpp")
PROBE_BYTES = 2 * 1024 ** 3


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name):
    """'void gf::k_update_half<double, 6, 0, gf::UpdOR<double>, 4, true, false>(...)'
    -> 'k_update_half<double,6,0,UpdOR,4,true,false>'"""
    n = re.sub(r"\(.*$", "", name.replace("void ", "")).replace("gf::", "").replace("gen::", "")
    n = re.sub(r"UpdOR<\w+>", "UpdOR", n)
    n = re.sub(r"UpdHB<\w+>", "UpdHB", n)
    n = re.sub(r"UpdMicro<\w+>", "UpdMicro", n)
    n = re.sub(r"UpdORForm<\w+>", "UpdORForm", n)
    n = re.sub(r"UpdSR<\w+>", "UpdSR", n)
    return n.replace(" ", "")


def sweep_bytes(name, V):
    """Algorithmic bytes per launch of a half-sweep (overrelaxation, heatbath or
    microcanonical; one lattice or a batch of lattices of V sites in all): V/2
    sites, each reading and writing 8 links of R reals of b bytes, and g (12
    reals) read and written where it is tracked."""
    m = (re.match(r"k_update_half<(float|double),(\d+),\d+,Upd(?:OR|HB|Micro),\d+,\w+,(\w+)>", name)
         or re.match(r"k_update_half_batch<(float|double),(\d+),Upd(?:OR|HB|Micro),\d+,\w+,(\w+)>", name))
    if not m:
        return None
    b = 4 if m.group(1) == "float" else 8
    R = 2 * int(m.group(2))
    tracked = m.group(3) == "true"
    per_site = 16 * R * b + (2 * 12 * b if tracked else 0)
    return (V // 2) * per_site


def cmd_kernels(args):
    rows = list(csv.DictReader(open(args.csv)))
    print(f"# {args.title}\n")
    print(f"Command: `{args.command}`\n")
    print(f"Kernel sources hash: `{kernel_source_hash()}`\n")
    print("| kernel | calls | avg us | min us | max us | % time |")
    print("|---|---:|---:|---:|---:|---:|")
    for r in rows:
        print(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
              f"{float(r['Percentage']):.2f} |")


def _avg_counter(path):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}, {k: len(v) for k, v in agg.items()}


def cmd_counters(args):
    fetch, nf = _avg_counter(args.fetch)
    write, nw = _avg_counter(args.write)
    copy = [k for k in fetch if k.startswith("k_probe_copy")][0]
    f_scale = PROBE_BYTES / (fetch[copy] * 1024.0)
    w_scale = PROBE_BYTES / (write[copy] * 1024.0)
    V = 1
    for d in args.dims.split(","):
        V *= int(d)
    if args.sites:
        V = args.sites
    out = {"kernel_source_hash": kernel_source_hash(), "lattice": args.dims, "sites": V,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}}
    print(f"# {args.title}\n")
    print(f"Commands:\n\n```\n{args.command}\n```\n")
    print(f"Kernel sources hash: `{out['kernel_source_hash']}`. "
          + (f"{V} sites in all.\n" if args.sites else f"Lattice {args.dims}.\n"))
    print(f"Calibration: the copy probe moves 2 GiB in and 2 GiB out per dispatch; FETCH_SIZE "
          f"reads {fetch[copy]:.0f} KiB and WRITE_SIZE {write[copy]:.0f} KiB for it, so the "
          f"counters are scaled by {f_scale:.4f} and {w_scale:.4f}.\n")
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) | "
          "algorithmic bytes | ratio |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for k in fetch:
        if k not in write:
            continue
        tot = fetch[k] * 1024 * f_scale + write[k] * 1024 * w_scale
        alg = sweep_bytes(k, V)
        ratio = f"{tot / alg:.4f}" if alg else ""
        print(f"| `{k}` | {nf[k]} | {fetch[k]:.1f} | {write[k]:.1f} | {tot:.4g} | "
              f"{alg if alg else ''} | {ratio} |")
        out["kernels"][k] = {"traffic_bytes": tot, "algorithmic_bytes": alg}
    print("\n```json")
    print(json.dumps(out, indent=1))
    print("```")


def cmd_busy(args):
    rows = []
    with open(args.csv) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"])))
    rows.sort()
    pat = re.compile(args.match)
    split = args.split_ms * 1e6
    # stretches: maximal runs of kernels whose idle gaps are all below split
    stretches, cur, end = [], [], 0
    for a, b, n in rows:
        if cur and a - end > split:
            stretches.append(cur)
            cur = []
        end = b if not cur else max(end, b)
        cur.append((a, b, n))
    if cur:
        stretches.append(cur)
    print(f"# {args.title}\n")
    print(f"Command: `{args.command}`\n")
    print(f"Kernel sources hash: `{kernel_source_hash()}`\n")
    print(f"Stretches of GPU work split at idle gaps over {args.split_ms} ms; listed: those with a "
          f"kernel matching `{args.match}`. Busy: the union of kernel intervals.\n")
    print("| stretch | wall ms | kernels | matching | busy ms | busy % | gaps > 5 us | idle in them ms | "
          "largest gap us |")
    print("|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
    out = []
    for i, st in enumerate(stretches):
        m = sum(1 for _, _, n in st if pat.search(n))
        if not m:
            continue
        busy, gaps, idle, big, hi = 0, 0, 0, 0, None
        for a, b, _ in st:
            if hi is None:
                busy, hi = b - a, b
                continue
            if a > hi:
                g = a - hi
                if g > 5000:
                    gaps += 1
                    idle += g
                big = max(big, g)
                busy += b - a
                hi = b
            elif b > hi:
                busy += b - hi
                hi = b
        wall = hi - st[0][0]
        out.append({"wall_ms": wall / 1e6, "busy_frac": busy / wall})
        print(f"| {i} | {wall / 1e6:.1f} | {len(st)} | {m} | {busy / 1e6:.1f} | {100 * busy / wall:.2f} | "
              f"{gaps} | {idle / 1e6:.2f} | {big / 1e3:.1f} |")
    print("\n```json")
    print(json.dumps({"stretches": out}, indent=1))
    print("```")


def load_counters(path):
    """The JSON block of a `counters` summary, or None."""
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    return json.loads(m.group(1)) if m else None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("csv")
    k.add_argument("--command", required=True)
    k.add_argument("--title", default="Kernel trace")
    c = sub.add_parser("counters")
    c.add_argument("fetch")
    c.add_argument("write")
    c.add_argument("--command", required=True)
    c.add_argument("--dims", default="32,32,32,32")
    c.add_argument("--sites", type=int, default=0, help="sites in all (a batch), instead of --dims")
    c.add_argument("--title", default="HBM counters")
    b = sub.add_parser("busy")
    b.add_argument("csv")
    b.add_argument("--match", required=True)
    b.add_argument("--split-ms", type=float, default=20.0)
    b.add_argument("--command", required=True)
    b.add_argument("--title", default="GPU busy time")
    args = ap.parse_args(argv)
    {"kernels": cmd_kernels, "counters": cmd_counters, "busy": cmd_busy}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
