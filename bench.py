#!/usr/bin/env python3
"""Benchmark: two-stage s-step GMRES on one MI355X.

One step = one full solve of the 2D Laplace 5-point system on a 2048 x 2048 grid
(n = 4,194,304, CSR float64), b = A x_true with x_true ~ U(-1,1) (seed 0), x0 = 0,
restart m = 60, step s = 5, two-stage block orthogonalization (s_hat = m),
relative residual 1e-10.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  value = solves per second (whole job, one GPU).  Extra fields:
time to solution, per-kernel-class times from HIP events recorded by the library on
the solve's stream, the roofline of the dominant kernel, the isolated block
orthogonalization of a 4,194,304 x 61 float64 Gaussian block, and the FP64 CPU
oracle timed on a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ortho time & time-to-solution (2D Laplace n=4M) + HBM GB/s; solves/s, p99"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kernel_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2402_15033_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hpp", ".hip")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel sources (else None)."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


# kernel classes that make up the orthogonalization (every class the library times except
# the SpMV, the residual, the first-vector scaling, the x update and the preconditioner)
ORTHO_CLASSES = ("gram", "gram_first", "update", "fused", "tail", "cycle_end", "fallback", "stage2")

METHOD_PASSES_DOC = {
    "two_stage": "sum_j (2 k_j + 3 s) + (m + 1) column passes per cycle (stage 1 per panel; the stage-2 "
                 "Gram read, its explicit Q folded into the x update), k_j = (j - 1) s + 1",
    "bcgs_pip2": "sum_j 2 (2 k_j + 3 s) column passes per cycle",
    "bcgs2_cholqr2": "sum_j (4 k_j + 15 s) column passes per cycle",
    "cgs2": "sum_{k=1..m} (4 k + 9) column passes per cycle",
}


def method_column_passes(ortho: str, m: int, s: int) -> int:
    """Column passes (reads + writes of one n-vector) of one restart cycle of the method's
    orthogonalization, the byte model of the measurement plan."""
    if ortho == "cgs2":
        return sum(4 * k + 9 for k in range(1, m + 1))
    ks = [j * s + 1 for j in range(m // s)]
    if ortho == "two_stage":
        return sum(2 * k + 3 * s for k in ks) + (m + 1)
    if ortho == "bcgs_pip2":
        return sum(2 * (2 * k + 3 * s) for k in ks)
    return sum(4 * k + 15 * s for k in ks)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _counter_rows(d: str):
    """(kernel name, dispatch id, counter value) of a rocprofv3 --pmc csv run in directory d."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {d}")
    out = []
    for f in files:
        for r in csv.DictReader(open(f)):
            out.append((r["Kernel_Name"], int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    return out


def _kernel_key(name: str) -> str:
    """The name the bench uses for a kernel: a batched body's own name (MpkBody<double, double,
    1>), else the kernel's signature without its return type."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    pre = "tsg::batched_kernel<tsg::"
    if name.startswith(pre):
        body = name[len(pre):name.index(">(")].strip()
        return body[:-1].strip() if body.endswith(">") and body.count("<") < body.count(">") else body
    return name


def write_traffic(fetch_dir: str, write_dir: str):
    """HBM bytes per launch of every kernel of the --pmc-probe run, from its FETCH_SIZE and
    WRITE_SIZE counter runs (KiB per dispatch, paired by dispatch id: both runs launch the
    same sequence), each scaled by what the counter reads for the probe's 1 GiB device copies
    (the calibration copies of known size: the copy dispatches that write at least half a
    GiB).  Dispatches that did no work (gated launches that return at entry: below 1% of the
    kernel's largest) are dropped.  Writes profiles/kernel_traffic.json with the hash of the
    kernel sources it was taken on, and prints the table as markdown."""
    runs = []
    for d in (fetch_dir, write_dir):
        per = {}
        for name, disp, v in _counter_rows(d):
            per[disp] = (_kernel_key(name), per.get(disp, (None, 0.0))[1] + v)
        runs.append(per)
    fetch, write = runs
    agg = {}
    for disp, (name, fv) in fetch.items():
        if disp in write and write[disp][0] == name:
            agg.setdefault(name, []).append((fv, write[disp][1]))
    copy = [k for k in agg if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no calibration copy in the counter runs")
    cal_kb = (1 << 30) / 1024.0
    cp = agg[copy[0]]
    wmax = max(w for _, w in cp)
    big = [(f, w) for f, w in cp if w >= 0.5 * wmax]
    ff = cal_kb / (sum(f for f, _ in big) / len(big))
    wf = cal_kb / (sum(w for _, w in big) / len(big))
    kernels = {}
    for name, v in agg.items():
        if name in copy:
            continue
        top = max(f for f, _ in v)
        keep = [(f, w) for f, w in v if f >= 0.01 * top] if top > 0 else v
        fkb = sum(f for f, _ in keep) / len(keep)
        wkb = sum(w for _, w in keep) / len(keep)
        kernels[name] = {"dispatches": len(keep), "fetch_kb": round(fkb, 1), "write_kb": round(wkb, 1),
                         "hbm_bytes_per_launch": int(round(1024 * (fkb * ff + wkb * wf)))}
    rec = {"source_hash": kernel_source_hash(),
           "commands": ["rocprofv3 --pmc FETCH_SIZE -d " + fetch_dir + " -o run --output-format csv -- python3 bench.py --pmc-probe",
                        "rocprofv3 --pmc WRITE_SIZE -d " + write_dir + " -o run --output-format csv -- python3 bench.py --pmc-probe"],
           "copy_calibration": {"bytes": 1 << 30, "copies": len(big),
                                "fetch_kb": round(sum(f for f, _ in big) / len(big), 1),
                                "write_kb": round(sum(w for _, w in big) / len(big), 1),
                                "fetch_factor": round(ff, 4), "write_factor": round(wf, 4)},
           "kernels": dict(sorted(kernels.items(), key=lambda kv: -kv[1]["hbm_bytes_per_launch"] * kv[1]["dispatches"]))}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("| kernel | dispatches | FETCH_SIZE KB | WRITE_SIZE KB | HBM bytes / launch |")
    print("|---|---:|---:|---:|---:|")
    for name, k in rec["kernels"].items():
        print(f"| `{name.split('(')[0]}` | {k['dispatches']} | {k['fetch_kb']} | {k['write_kb']} | {k['hbm_bytes_per_launch']:,} |")

def np_mean(v):
    return sum(v) / len(v)


def ortho_bench(args, tsg, W, np, torch, dev, n):
    """The isolated two-stage block orthogonalization of a Gaussian n x 61 block (s = args.s,
    one big panel), median over args.ortho_reps calls, at ld = n + 512 and ld = n."""
    k, s = 61, args.s
    log(f"[bench] isolated block orthogonalization {n} x {k}")
    X0 = torch.as_tensor(W.gaussian_block(n, k, seed=7).T.copy(), device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for pad in (512, 0):
        # columns n + 512 elements apart (the solver's basis layout: column starts that are
        # multiples of 64 Ki elements put the columns on the same HBM channels), and the
        # unpadded layout for reference
        buf = torch.empty((k, n + pad), dtype=torch.float64, device=dev)
        Xw = buf[:, :n]
        times = []
        for r in range(args.ortho_reps + 2):
            Xw.copy_(X0)
            e0.record()
            tsg.orthogonalize(Xw, s=s, algo="two_stage")
            e1.record()
            torch.cuda.synchronize()
            if r >= 2:
                times.append(e0.elapsed_time(e1))
        res[pad] = float(np.median(times))
        if pad == 512:
            _, _, oerr = tsg.orthogonalize(Xw.copy_(X0), s=s, algo="two_stage", orth_err=True)
        del buf, Xw
    med = res[512]
    # context: torch's own kernels on the same padded block, a read-only reduction over the
    # rows of every column and an in-place scaling (every column read and written once)
    buf = torch.empty((k, n + 512), dtype=torch.float64, device=dev)
    Xw = buf[:, :n]
    Xw.copy_(X0)
    ctx = {}
    for name, fn, passes_ in (("torch_column_sums", lambda: Xw.sum(dim=1), k),
                              ("torch_inplace_scale", lambda: Xw.mul_(1.0), 2 * k)):
        ts = []
        for r in range(7):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if r >= 2:
                ts.append(e0.elapsed_time(e1))
        ctx[name + "_GBps"] = round(passes_ * n * 8 / float(np.median(ts)) / 1e6, 1)
    del buf, Xw
    passes = 1047 if (args.s == 5 and k == 61) else None
    method_bytes = sum(2 * c0 + 3 * min(s, k - c0) for c0 in range(1, k, s)) * n * 8 + 3 * k * n * 8
    return {"shape": [n, k], "ld": n + 512, "s": s, "algo": "two_stage", "median_ms": round(med, 3),
            "median_ms_ld_n": round(res[0], 3),
            "method_column_passes": passes if passes else round(method_bytes / (n * 8)),
            "method_GB": round(method_bytes / 1e9, 3),
            "GBps": round(method_bytes / med / 1e6, 1),
            "frac": round(method_bytes / med / 1e6 / HBM_PEAK_GBPS, 4),
            "byte_model": "stage 1 sum_j (2 k_j + 3 s) + stage 2 3 k column passes (Gram read, "
                          "explicit Q read and written)",
            "orth_err": oerr, "reps": args.ortho_reps, "context": ctx}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--problem", default="laplace2d", choices=["laplace2d", "laplace3d", "convdiff2d"])
    ap.add_argument("--N", type=int, default=None,
                    help="grid side (default 2048 in 2D, 160 in 3D)")
    ap.add_argument("--basis", default="monomial", choices=["monomial", "shifted", "leja"])
    ap.add_argument("--precond", default="none", choices=["none", "mcgs"],
                    help="right preconditioning: multicolor Gauss-Seidel (the workload of Fig. 13)")
    ap.add_argument("--s-hat", type=int, default=0, help="two-stage big-panel size (0 = m)")
    ap.add_argument("--shat-sweep", action="store_true",
                    help="also time one solve for each s_hat in {s, 2s, 4s, 6s, m} (Table 2's knob)")
    ap.add_argument("--s", type=int, default=5)
    ap.add_argument("--m", type=int, default=60)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--ortho", default="two_stage",
                    choices=["two_stage", "bcgs_pip2", "bcgs2_cholqr2", "cgs2"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_ir"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ortho-bench", action="store_true")
    ap.add_argument("--ortho-only", action="store_true",
                    help="only the isolated block orthogonalization (n = N^2 rows, 61 columns)")
    ap.add_argument("--ortho-reps", type=int, default=20)
    ap.add_argument("--cpu-budget-s", type=float, default=30.0,
                    help="host seconds for the CPU oracle legs (all cores, then one thread)")
    ap.add_argument("--time-stride", type=int, default=16,
                    help="HIP-event timing of every launch in every n-th restart cycle of the timed "
                         "solves (1 = every cycle; events between launches slow a cycle by ~12%%)")
    ap.add_argument("--eager", action="store_true",
                    help="launch every kernel directly instead of replaying one captured cycle")
    ap.add_argument("--modes", action="store_true",
                    help="also time one solve in each launch mode (graph/eager x events on/off)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/kernel_traffic.json (and print its table) from the two rocprofv3 "
                         "counter runs of --pmc-probe: FETCH_SIZE in FETCH_DIR, WRITE_SIZE in WRITE_DIR")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short run for hardware-counter passes: three 1 GiB device copies (the "
                         "calibration kernel) and the first two restart cycles of the solve")
    ap.add_argument("--serve", action="store_true",
                    help="run the served form instead: Poisson arrivals of mixed solves through the "
                         "continuous-batching server")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-seed", type=int, default=0)
    ap.add_argument("--serve-sides", default="128,256,512,1024,2048",
                    help="grid sides the served requests draw from (uniformly)")
    ap.add_argument("--compare", action="store_true",
                    help="also time one solve of each other orthogonalization scheme")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(*args.traffic_from)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on exactly one GPU (the whole problem fits one MI355X); "
              "multi-GPU runs are not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2402_15033_amd as tsg
    import workloads as W

    dev = torch.device("cuda:0")
    tsg.load_library()
    if args.serve:
        serve_bench(args, tsg, W, np, torch, dev)
        return
    if args.pmc_probe:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        N = args.N or 2048
        pr = W.make_problem(args.problem, N, seed=0)
        A = tsg.CSRMatrix.from_host(pr["A"], device=dev)
        b = torch.as_tensor(pr["b"], device=dev)
        _, info = tsg.solve(A, b, m=args.m, s=args.s, tol=args.tol, ortho=args.ortho,
                            precision=args.precision, basis=args.basis, max_iters=2 * args.m, graph=False)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": True, "copy_bytes": 1 << 30, "iters": int(info.iters)}), flush=True)
        return
    N = args.N or (160 if args.problem == "laplace3d" else 2048)
    if args.ortho_only:
        ob = ortho_bench(args, tsg, W, np, torch, dev, N * N)
        print(json.dumps({"ortho_bench": ob}), flush=True)
        return
    desc = {"laplace2d": f"2D Laplace 5-point {N}x{N}", "laplace3d": f"3D Laplace 7-point {N}^3",
            "convdiff2d": f"2D convection-diffusion upwind {N}x{N}"}[args.problem]
    log(f"[bench] building {desc}")
    pr = W.make_problem(args.problem, N, seed=0)
    if args.problem == "convdiff2d":
        desc += f" (Pe={pr['meta']['pe']:.2f}, theta={pr['meta']['theta']:.3f})"
    Ah = pr["A"]
    A = tsg.CSRMatrix.from_host(Ah, device=dev)
    precond = None if args.precond == "none" else args.precond
    if precond:
        A.precond_setup()
        desc += f", multicolor Gauss-Seidel ({A.ncolors} colors)"
    b = torch.as_tensor(pr["b"], device=dev)
    x = torch.zeros_like(b)
    kw = dict(m=args.m, s=args.s, tol=args.tol, ortho=args.ortho, precision=args.precision,
              basis=args.basis, graph=not args.eager, s_hat=args.s_hat, precond=precond)
    need = tsg.binding.solve_workspace_bytes(A, m=args.m, s=args.s, ortho=args.ortho,
                                             precision=args.precision, s_hat=args.s_hat, precond=precond)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:]
    torch.cuda.synchronize()

    for i in range(args.warmup):
        x.zero_()
        _, info = tsg.solve(A, b, x, workspace=ws, **kw)
        log(f"[bench] warmup {i}: iters={info.iters} cycles={info.cycles} relres={info.relres:.3e}")
    torch.cuda.synchronize()

    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        x.zero_()
        _, info = tsg.solve(A, b, x, workspace=ws, timing=args.time_stride, **kw)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} solves in {elapsed:.3f}s")
    info = infos[-1]
    # independent residual check of the final iterate (scipy on the host)
    xh = x.cpu().numpy()
    relres_host = float(np.linalg.norm(pr["b"] - Ah.to_scipy() @ xh) / np.linalg.norm(pr["b"]))
    if not info.converged:
        log(f"[bench] WARNING: the solve did not converge (status {info.status}, relres {relres_host:.3e})")

    def tot(f):
        return sum(getattr(i, f) for i in infos)

    tcyc = tot("timed_cycles")

    # per kernel class (one kernel instantiation each), from HIP events on the solve stream
    classes = {}
    for inf in infos:
        for name, (cms, cn, cby) in inf.kernel_classes().items():
            a = classes.setdefault(name, [0.0, 0, 0.0])
            a[0] += cms
            a[1] += cn
            a[2] += cby
    elem = "double" if args.precision == "fp64" else "float"
    st_ = lambda w: w if w <= 6 else (8 if w <= 8 else (10 if w <= 10 else (12 if w <= 12 else 16)))
    s_ = args.s
    nt2 = 1 if 2 * args.s <= 16 else 2
    # the packed operator stores column - row in 16 bits when every delta of the matrix fits
    rows = np.repeat(np.arange(Ah.n, dtype=np.int64), np.diff(Ah.row_ptr))
    delta = Ah.col.astype(np.int64) - rows
    fmt = 1 if Ah.nnz == 0 or (delta.min() >= -32768 and delta.max() <= 32767) else 2  # 16- or 32-bit
    names = {  # every per-request kernel runs as batched_kernel<Body>
        "mpk": f"MpkBody<{elem}, {elem}, {fmt}>",
        "gram": f"GramBody<{elem}, 1..5, {nt2}>",
        "gram_first": f"GramBody<{elem}, 1..2, 1..2>",
        "update": f"UpdateBody<{elem}, {st_(s_)}, 128>",
        "fused": f"FusedBody<{elem}, 4>",
    }
    streaming = {c: v for c, v in classes.items() if c in names and v[0] > 0}
    dom = max(streaming, key=lambda c: streaming[c][0])
    ms, cnt, by = streaming[dom]
    kname = names[dom]
    w = 8.0 if args.precision == "fp64" else 4.0
    per_launch_us = ms / cnt * 1e3
    format_bytes = by / cnt  # the library's own count for the launched layout
    # the survey's per-launch byte model: a CSR SpMV step reads w + 4 bytes per stored entry,
    # the row pointers and x once, and writes y; the panel kernels' algorithmic bytes are
    # the w n (columns read + written) the library counts
    if dom == "mpk":
        model_bytes = (w + 4.0) * Ah.nnz + 4.0 * (Ah.n + 1) + 2.0 * w * Ah.n
        model = "CSR SpMV step: (w + 4) nnz + 4 (n + 1) + 2 w n bytes (w = element bytes)"
    else:
        model_bytes = format_bytes
        model = "w n (columns read + columns written)"
    achieved = model_bytes / (per_launch_us * 1e-6) / 1e9
    traffic = measured_traffic(kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": traffic, "kernel": kname,
                "byte_model": model, "algorithmic_bytes_per_launch": round(model_bytes),
                "avg_launch_us": round(per_launch_us, 2), "launches": int(cnt),
                "time_source": (f"HIP events around every launch of every {args.time_stride}th restart cycle "
                                "of the timed solves (launched directly), on the solve's stream; they include "
                                "the launch gap"),
                "format_bytes_per_launch": round(format_bytes),
                "frac_format": round(format_bytes / (per_launch_us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4),
                "frac_counter": (round(traffic / (per_launch_us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4)
                                 if traffic else None),
                "timed_cycles": int(tcyc), "time_stride": args.time_stride}
    per_class = {}
    for c, (cms, ccnt, cby) in classes.items():
        per_class[c] = {"kernel": names.get(c), "ms_per_cycle": round(cms / tcyc, 4),
                        "launches_per_cycle": round(ccnt / tcyc, 2),
                        "GBps": round(cby / (cms * 1e-3) / 1e9, 1) if cms > 0 and cby > 0 else None}
    ortho_ms_cycle = sum(classes[c][0] for c in ORTHO_CLASSES if c in classes) / tcyc
    passes = method_column_passes(args.ortho, args.m, args.s)
    ortho_gb = passes * Ah.n * w / 1e9
    ortho = {"ms_per_cycle": round(ortho_ms_cycle, 3), "classes": [c for c in ORTHO_CLASSES if c in classes],
             "column_passes_per_cycle": passes, "method_GB_per_cycle": round(ortho_gb, 3),
             "GBps": round(ortho_gb / (ortho_ms_cycle * 1e-3), 1),
             "frac": round(ortho_gb / (ortho_ms_cycle * 1e-3) / HBM_PEAK_GBPS, 4),
             "byte_model": METHOD_PASSES_DOC.get(args.ortho)}

    out = {
        "metric": METRIC,
        "value": round(args.steps / elapsed, 5),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{desc} (n={Ah.n}, nnz={Ah.nnz}) CSR, "
                               f"x_true~U(-1,1) seed 0, x0=0; s-step GMRES m={args.m} s={args.s} "
                               f"{args.ortho} (s_hat={args.s_hat or args.m}), {args.basis} basis, tol={args.tol:g}, "
                               f"{args.precision}",
                   "problem": args.problem, "N": N,
                   "n": Ah.n, "nnz": Ah.nnz, "m": args.m, "s": args.s, "ortho": args.ortho,
                   "basis": args.basis, "precision": args.precision, "tol": args.tol,
                   "precond": args.precond,
                   "s_hat": args.s_hat or args.m},
        "time_to_solution_s": round(elapsed / args.steps, 4),
        "iters": int(info.iters), "cycles": int(info.cycles),
        "relres_device": info.relres, "relres_host_check": relres_host,
        "converged": bool(info.converged), "status": int(info.status),
        "pip_fallbacks": int(info.pip_fallbacks), "shifted_passes": int(info.shifted_passes),
        "newton_from_cycle": int(info.newton_from_cycle),
        "ortho_ms_per_cycle": round(ortho_ms_cycle, 3),
        "ortho": ortho,
        "kernel_classes": per_class,
        "roofline": roofline,
    }

    if args.modes:
        modes = {}
        for graph in (True, False):
            for timing in (False, True):
                x.zero_()
                torch.cuda.synchronize()
                t = time.perf_counter()
                key = ("graph" if graph else "eager") + ("+events" if timing else "")
                try:
                    tsg.solve(A, b, x, workspace=ws, timing=int(timing), **dict(kw, graph=graph))
                except tsg.TSGError as exc:
                    modes[key] = str(exc)
                    log(f"[bench] mode {key}: {exc}")
                    continue
                torch.cuda.synchronize()
                modes[key] = round(time.perf_counter() - t, 4)
                log(f"[bench] mode {key}: {modes[key]} s")
        out["launch_modes_s"] = modes

    if args.shat_sweep and args.ortho == "two_stage":
        sweep = {}
        for sh in sorted({args.s, 2 * args.s, 4 * args.s, 6 * args.s, args.m}):
            if sh > args.m or args.m % sh:
                continue
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, si = tsg.solve(A, b, x, workspace=None, **dict(kw, s_hat=sh))
            torch.cuda.synchronize()
            sweep[sh] = {"time_to_solution_s": round(time.perf_counter() - t, 4), "iters": int(si.iters),
                         "cycles": int(si.cycles), "relres": si.relres}
            log(f"[bench] s_hat {sh}: {sweep[sh]}")
        out["s_hat_sweep"] = sweep

    if args.compare:
        cmp = {}
        for o in ("two_stage", "bcgs_pip2", "bcgs2_cholqr2", "cgs2"):
            if o == args.ortho:
                cmp[o] = {"time_to_solution_s": out["time_to_solution_s"], "iters": out["iters"],
                          "ortho_ms_per_cycle": out["ortho_ms_per_cycle"]}
                continue
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, ci = tsg.solve(A, b, x, workspace=None, timing=True, m=args.m, s=args.s, tol=args.tol,
                              ortho=o, precision=args.precision, basis=args.basis, graph=not args.eager,
                              precond=precond)
            torch.cuda.synchronize()
            t = time.perf_counter() - t
            kc = ci.kernel_classes()
            oms = sum(kc[c][0] for c in ORTHO_CLASSES if c in kc) / max(ci.timed_cycles, 1)
            cmp[o] = {"time_to_solution_s": round(t, 4), "iters": int(ci.iters), "relres": ci.relres,
                      "ortho_ms_per_cycle": round(oms, 3),
                      "ortho_frac": round(method_column_passes(o, args.m, args.s) * Ah.n * w / (oms * 1e-3)
                                          / 1e9 / HBM_PEAK_GBPS, 4)}
            log(f"[bench] compare {o}: {cmp[o]}")
        out["compare"] = cmp

    if args.precision == "fp32_ir":
        # the mixed form's error per solve against the plain FP64 solve of the same system
        xr = torch.zeros_like(b)
        _, i64 = tsg.solve(A, b, xr, **dict(kw, precision="fp64"))
        torch.cuda.synchronize()
        x64 = xr.cpu().numpy()
        xt = pr.get("x_true")
        out["vs_fp64"] = {"rel_diff_x": float(np.linalg.norm(xh - x64) / np.linalg.norm(x64)),
                          "fp64_iters": int(i64.iters), "fp64_relres": i64.relres,
                          "rel_err_mixed_vs_x_true": (float(np.linalg.norm(xh - xt) / np.linalg.norm(xt))
                                                      if xt is not None else None),
                          "rel_err_fp64_vs_x_true": (float(np.linalg.norm(x64 - xt) / np.linalg.norm(xt))
                                                     if xt is not None else None)}
        log(f"[bench] mixed vs FP64: {out['vs_fp64']}")

    if not args.no_ortho_bench:
        out["ortho_bench"] = ortho_bench(args, tsg, W, np, torch, dev, Ah.n)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, Ah, pr, info, desc, precond)
    print(json.dumps(out), flush=True)


def cpu_baseline(args, Ah, pr, info, desc, precond):
    """The FP64 oracle on the host cores, on a bounded sample of the same solve: restart
    cycles timed with all the cores numpy's BLAS uses and with one thread; the solve's time
    is extrapolated with the GPU's cycle count.  Each leg runs one cycle, then as many more
    as fit its budget (10 at most)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import gmres as G
    from oracle import precond as PC
    from oracle import sparse as S

    op = S.Operator(Ah)
    prec = PC.MulticolorGS(Ah) if precond else None
    ortho = args.ortho if args.ortho != "cgs2" else "two_stage"

    def run(cycles):
        t = time.perf_counter()
        ref = G.sstep_gmres(op, pr["b"], m=args.m, s=args.s, tol=args.tol, ortho=ortho, basis=args.basis,
                            max_iters=cycles * args.m, precond=prec)
        return time.perf_counter() - t, ref["cycles"]

    def leg(budget):
        t1, c1 = run(1)
        more = int(min(9, max(0, budget / max(t1, 1e-9) - 1)))
        if more == 0:
            return t1 / max(c1, 1), c1
        t2, c2 = run(more)
        return t2 / max(c2, 1), c2

    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    log(f"[bench] CPU oracle, {threads} threads")
    t_all, c_all = leg(args.cpu_budget_s / 2)
    log(f"[bench] CPU oracle, 1 thread")
    with threadpool_limits(limits=1):
        t_one, c_one = leg(args.cpu_budget_s / 2)
    cyc = max(info.cycles, 1)
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:
        avail = os.cpu_count()
    return {"value": 1.0 / (t_all * cyc), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"restart cycles of the same {desc} solve, timed and scaled by the {cyc} cycles the GPU "
                       f"solve needed: all-core leg {c_all} cycle(s) at {t_all:.2f} s/cycle (numpy BLAS on "
                       f"{threads} threads, scipy SpMV single-threaded), single-thread leg {c_one} cycle(s) "
                       f"at {t_one:.2f} s/cycle"),
            "single_thread": {"value": 1.0 / (t_one * cyc), "s_per_cycle": round(t_one, 3), "cycles_timed": c_one},
            "all_cores": {"value": 1.0 / (t_all * cyc), "s_per_cycle": round(t_all, 3), "cycles_timed": c_all,
                          "threads": threads},
            "cpu_model": cpu_model(), "host_cpus_available": avail}


def serve_bench(args, tsg, W, np, torch, dev):
    """The served form: a seeded Poisson stream of solves with grid sides uniform in
    {128, ..., 2048}, half 2D Laplace and half convection-diffusion (Pe ~ U[1,100]),
    b ~ U(-1,1), m = 60, s = 5, FP32 basis with FP64 refinement, tol 1e-8, admitted
    against an HBM budget by the continuous-batching server.  Inputs are built and
    resident on the device before the clock starts; latency = completion - arrival
    (queueing included)."""
    rng = np.random.default_rng(args.serve_seed)
    R = args.serve_requests
    gaps = rng.exponential(1.0 / args.serve_rate, size=R)
    arrival = np.cumsum(gaps) - gaps[0]
    side_set = [int(v) for v in args.serve_sides.split(",")]
    sides = rng.choice(side_set, size=R)
    kinds = np.where(rng.random(R) < 0.5, "laplace2d", "convdiff2d")
    log(f"[serve] building {R} requests")
    reqs = []
    lap_cache = {}
    for i in range(R):
        kind, N = str(kinds[i]), int(sides[i])
        pr = W.make_problem(kind, N, seed=1000 + i, rhs="uniform", pe_range=(1.0, 100.0))
        if kind == "laplace2d" and N in lap_cache:
            A = lap_cache[N]
        else:
            A = tsg.CSRMatrix.from_host(pr["A"], device=dev)
            if kind == "laplace2d":
                lap_cache[N] = A
        b = torch.as_tensor(pr["b"], device=dev)
        reqs.append({"kind": kind, "N": N, "A": A, "b": b, "n": pr["A"].n})
        if (i + 1) % 100 == 0:
            log(f"[serve] built {i + 1}/{R}")
    torch.cuda.synchronize()
    srv = tsg.Server(int(args.serve_budget_gb * 2**30), m=args.m, s=args.s, tol=1e-8, basis="shifted",
                     precision="fp32_ir", max_active=256, device=dev)
    log("[serve] running")
    done = {}
    nxt = 0
    max_active = 0
    steps = 0
    t0 = time.perf_counter()
    last_log = t0
    while len(done) < R:
        now = time.perf_counter() - t0
        while nxt < R and arrival[nxt] <= now:
            r = reqs[nxt]
            r["x"] = srv.submit(nxt, r["A"], r["b"])
            nxt += 1
        na, nq = srv.step()
        steps += 1
        max_active = max(max_active, na)
        t = time.perf_counter() - t0
        for tag, x, info in srv.poll():
            done[tag] = (t, info)
        if na == 0 and nq == 0 and nxt < R and len(done) < R:
            time.sleep(max(0.0, arrival[nxt] - (time.perf_counter() - t0)))
        if time.perf_counter() - last_log > 20:
            last_log = time.perf_counter()
            log(f"[serve] t={t:.1f}s done {len(done)}/{R} active {na} queued {nq}")
    makespan = time.perf_counter() - t0
    lat = np.array([done[i][0] - arrival[i] for i in range(R)])
    conv = sum(1 for i in range(R) if done[i][1].status == 0)
    iters = [int(done[i][1].iters) for i in range(R)]
    per = {}
    for i in range(R):
        key = f"{reqs[i]['kind']}_{reqs[i]['N']}"
        per.setdefault(key, []).append(float(lat[i]))
    out = {
        "metric": "served solves/s and p50/p99 latency (Poisson mix of 2D Laplace / convection-diffusion "
                  f"{min(side_set)}^2..{max(side_set)}^2, FP32+FP64 refinement, tol 1e-8)",
        "value": round(R / makespan, 4), "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals, grid side uniform in {{{args.serve_sides}}}, half 2D Laplace "
                               "and half upwind convection-diffusion (Pe~U[1,100]), b~U(-1,1), m=60, s=5, "
                               "two-stage, shifted basis, FP32 basis + FP64 refinement, tol 1e-8",
                   "requests": R, "arrival_rate_per_s": args.serve_rate, "hbm_budget_gb": args.serve_budget_gb,
                   "seed": args.serve_seed},
        "makespan_s": round(makespan, 3),
        "offered_load_per_s": args.serve_rate,
        "achieved_solves_per_s": round(R / makespan, 4),
        "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
        "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
        "latency_max_s": round(float(lat.max()), 3),
        "converged": conv, "total_iterations": int(sum(iters)), "cycles_run": steps,
        "max_active": max_active,
        "latency_p50_by_kind_size_s": {k: round(float(np.median(v)), 3) for k, v in sorted(per.items())},
    }
    srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
