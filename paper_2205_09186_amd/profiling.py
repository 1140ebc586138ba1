"""Workload driver and summariser for rocprofv3 runs of the step kernels.

``python3 -m paper_2205_09186_amd.profiling run`` performs one plain 1 GiB
device-to-device copy (the calibration kernel: 1 GiB read, 1 GiB written) and
then a few steps of the benchmark workload (or, with --probe, a few launches of
the population copy that measures the access pattern's ceiling; with --batch,
a few steps of the batched sweep on the config-3 set), so one rocprofv3 run
covers both.

``python3 -m paper_2205_09186_amd.profiling summarize --fetch DIR --write DIR
--trace DIR`` reads the CSV output of the counter runs (FETCH_SIZE, then
WRITE_SIZE, KiB per dispatch) and of a kernel-trace run, scales each counter by
what it reads for the calibration copy, and writes ``profiles/traffic.json``
(consumed by bench.py, one entry per workload and kernel) plus a markdown
summary.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CALIB_BYTES = 1 << 30


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2205_09186_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload_name(lattice, n, Tr, scheme, k):
    dims = 3 if lattice == "D3Q19" else 2
    return f"{lattice} {n}^{dims} droplet R={0.25 * n:g} Tr={Tr} {scheme} k={k}"


def run(args):
    import torch
    from paper_2205_09186_amd import inputs, lbm
    src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    if args.batch is not None:
        # the config-3 set in one batch, every instance running, in the given
        # launch form (512-node blocks)
        from paper_2205_09186_amd import sweep
        _, params, rhos = sweep.build()
        b = lbm.Batch(params, rhos)
        b.set_block(512)
        b.set_form(lbm.BATCH_PHASES if args.batch == "phases" else lbm.BATCH_PERSISTENT)
        b.run(args.steps, check_every=100, tol=0.0, chunk=args.steps)
        torch.cuda.synchronize()
        print(f"profiled the config-3 batch, {args.batch} form, {args.steps} steps ({b.launch_mode})", flush=True)
        return
    lat = lbm.D3Q19 if args.lattice == "D3Q19" else lbm.D2Q9
    n = args.n
    shape = (n, n, n) if lat == lbm.D3Q19 else (n, n)
    if args.probe:
        # the population copy that bench.py reports as the ceiling of the
        # access pattern: aligned, then as the pull, args.steps launches each
        import ctypes as C
        nz = n if lat == lbm.D3Q19 else 1
        q = 19 if lat == lbm.D3Q19 else 9
        a = torch.rand(q * n * n * nz, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        st = torch.cuda.current_stream()
        for pull in (0, 1):
            for _ in range(args.steps):
                lbm._check(lbm.lib().lbm_probe_copy(lat, n, n, nz, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                                    pull, C.c_void_p(st.cuda_stream)))
        torch.cuda.synchronize()
        print(f"profiled the {args.lattice} {n}^{len(shape)} population copy, {args.steps} launches each", flush=True)
        return
    p = lbm.Params(lattice=lat, nx=n, ny=n, nz=(n if lat == lbm.D3Q19 else 1), Tr=args.Tr, k=args.k,
                   kappa=args.kappa, scheme=lbm.SCHEMES[args.scheme])
    g, l = lbm.coexistence(args.Tr)
    sim = lbm.Simulation(p, torch.from_numpy(inputs.droplet(shape, 0.25 * n, 10.0, g, l).reshape(-1)).cuda())
    if args.variant is not None:
        names = [sim.variant_name(v) for v in range(sim.num_variants)]
        if args.variant not in names:
            sys.exit(f"no launch variant named {args.variant!r}; this workload has {names}")
        sim.set_variant(names.index(args.variant))
    sim.step(args.steps)
    torch.cuda.synchronize()
    print(f"profiled {workload_name(args.lattice, n, args.Tr, args.scheme, args.k)} variant {args.variant} "
          f"steps {args.steps}", flush=True)


def _rows(d, name):
    files = glob.glob(os.path.join(d, "**", f"*{name}*.csv"), recursive=True)
    out = []
    for f in files:
        with open(f) as fh:
            out.extend(csv.DictReader(fh))
    return out


def _counter_means(d, counter):
    """{kernel name: mean counter value per dispatch}"""
    acc = {}
    for r in _rows(d, "counter_collection"):
        if r.get("Counter_Name") != counter:
            continue
        k = r.get("Kernel_Name", "?")
        acc.setdefault(k, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _calibration(d, counter):
    """Counter value of the 1 GiB calibration copy: the largest copy dispatch."""
    vals = [float(r["Counter_Value"]) for r in _rows(d, "counter_collection")
            if r.get("Counter_Name") == counter and "copyBuffer" in r.get("Kernel_Name", "")]
    return max(vals) if vals else None


def _base(name: str) -> str:
    """Kernel name without return type, namespace, template arguments and
    parameter list ("void lbm::k_tile<1, 16, true, false>(...)" -> "k_tile")."""
    return name.split("<")[0].split("(")[0].replace("void ", "").replace("lbm::", "").strip()


def _match(means, key):
    """Counter mean of the kernel whose base name equals that of key (several
    instantiations of one kernel share it: their means are averaged)."""
    vals = [v for k, v in means.items() if _base(k) == _base(key)]
    if not vals:
        return None, None
    return _base(key), sum(vals) / len(vals)


def summarize(args):
    fetch = _counter_means(args.fetch, "FETCH_SIZE")
    write = _counter_means(args.write, "WRITE_SIZE")
    cf = _calibration(args.fetch, "FETCH_SIZE")
    cw = _calibration(args.write, "WRITE_SIZE")
    if cf is None or cw is None:
        sys.exit("calibration copy kernel not found in counter output")
    f_scale = (CALIB_BYTES / 1024.0) / cf
    w_scale = (CALIB_BYTES / 1024.0) / cw
    stats = _rows(args.trace, "kernel_stats")
    lines = ["# rocprofv3 summary: " + args.workload, "",
             "Commands (from the repository root, one run each):", "",
             "```", *args.commands.split(";"), "```", "",
             f"Calibration: 1 GiB device copy reads FETCH_SIZE {cf:.0f} KiB and WRITE_SIZE {cw:.0f} KiB; "
             f"scale factors {f_scale:.4f} (fetch), {w_scale:.4f} (write).", "",
             "| kernel | calls | avg duration (us) | FETCH KiB/dispatch | WRITE KiB/dispatch | scaled HBM bytes/dispatch |",
             "|---|---|---|---|---|---|"]
    rec = {}
    for r in stats:
        name = r.get("Name", "?")
        if "copyBuffer" in name:
            continue
        avg_us = float(r.get("AverageNs", 0)) / 1000.0
        _, fv = _match(fetch, name.split("(")[0])
        _, wv = _match(write, name.split("(")[0])
        scaled = None
        if fv is not None and wv is not None:
            scaled = (fv * f_scale + wv * w_scale) * 1024.0
        lines.append(f"| {name[:70]} | {r.get('Calls')} | {avg_us:.1f} | {fv if fv is None else round(fv)} | "
                     f"{wv if wv is None else round(wv)} | {scaled if scaled is None else round(scaled)} |")
        short = _base(name)
        if scaled is not None:
            rec[short] = {"avg_us": avg_us, "bytes": scaled}
    dom = args.kernel
    ent = rec.get(dom)
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(tpath)) if os.path.exists(tpath) else {}
    if ent:
        key = f"{args.workload} | {dom}" + (f" | variant {args.variant}" if args.variant is not None else "")
        data[key] = {"kernel": dom, "variant": args.variant, "bytes_per_launch": round(ent["bytes"]), "source_hash": source_hash(),
                               "avg_us_rocprof": round(ent["avg_us"], 2), "fetch_scale": round(f_scale, 5),
                               "write_scale": round(w_scale, 5)}
        json.dump(data, open(tpath, "w"), indent=1)
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--lattice", default="D3Q19")
    r.add_argument("--n", type=int, default=256)
    r.add_argument("--scheme", default="CD6")
    r.add_argument("--Tr", type=float, default=0.7)
    r.add_argument("--k", type=float, default=0.1)
    r.add_argument("--kappa", type=float, default=0.004)
    r.add_argument("--steps", type=int, default=5)
    r.add_argument("--variant", default=None,
                   help="launch variant by name, e.g. 'tile 64x16 z64' (default: the library's)")
    r.add_argument("--batch", choices=["phases", "persistent"], default=None,
                   help="profile the batched sweep on the config-3 set in this launch form instead")
    r.add_argument("--probe", action="store_true",
                   help="profile the population copy (lbm_probe_copy) on the grid instead of the step")
    s = sub.add_parser("summarize")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--trace", required=True)
    s.add_argument("--workload", required=True)
    s.add_argument("--kernel", default="k_ring")
    s.add_argument("--variant", default=None, help="name of the launch variant the counter runs used")
    s.add_argument("--commands", default="")
    s.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "run":
        run(a)
    else:
        summarize(a)


if __name__ == "__main__":
    main()
