#!/usr/bin/env python3
"""Benchmark of the hierarchical-probing hot path on one MI355X.

Workload: 4-D 32^4 torus, covariant Laplacian with 3 complex components per
site, Haar-random U(3) links, mass field m(x) = 0.1 + 0.02 clip(xi, +-3),
Z4 mask; 256 spatial probes x 3 diluted components = 768 CG solves to a true
relative residual of 1e-10 (FP64).  One step is one trace_inv_probe call over
all 768 right-hand sides, with the operator already resident on the GPU.
The headline value is the FP64 solver; the mixed-precision solver (FP32 CG,
FP64 reliable updates, same FP64 true-residual acceptance) is timed beside
it and reported under "mixed_precision", the same run with the gradient
of the last estimate (dT/dm and dT/dw, FP64) under "gradient", and the
batched solver on 64 uneven 3-D tori under "batch_c4".

Prints one JSON line: solves/s (the timed steps run as a user runs them,
chunks of CG iterations replayed as HIP graphs), the stencil kernel's
achieved HBM bandwidth against the MI355X peak (hipEvent timing of every
stencil launch in one more call with eager launches), and the CPU oracle
timed on a bounded sample of the same solve.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = [32, 32, 32, 32]
HBM_PEAK_GBS = 8000.0
METRIC = "probing-vector solves/sec (4D 32^4, rel.res 1e-10) + stencil HBM GB/s vs peak"
# the kernels and the host code that picks their launch shapes and tile order
KERNEL_SOURCES = ["paper_1302_4018_amd/csrc/tip_kernels.hip", "paper_1302_4018_amd/csrc/tip_device.h",
                  "paper_1302_4018_amd/csrc/tip_launch.h", "paper_1302_4018_amd/csrc/tip_kernel_common.h",
                  "paper_1302_4018_amd/csrc/tip_api.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stencil_traffic.json")
# the dominant kernel: with the even-odd reduction, the half-lattice stencil
# that forms S p (in FP64 in 512-thread workgroups unless TIP_EO_WIDE=0, in
# single precision with two rhs per thread unless TIP_EO_PAIR=0); without it,
# the 4-D marching stencil
STENCIL = {
    (True, "fp64"): ("k_eo_hop<tip::CovOp<HIP_vector_type<double, 2u> >, 1, 5, 256, false>" if os.environ.get("TIP_EO_WIDE") == "0"
                     else "k_eo_hop<tip::CovOp<HIP_vector_type<double, 2u> >, 1, 5, 512, false>"),
    (True, "fp32"): ("k_eo_hop<tip::CovOp<HIP_vector_type<float, 2u> >, 1, 5, 256, false>" if os.environ.get("TIP_EO_PAIR") == "0"
                     else "k_eo_hop_pair<tip::CovOp<HIP_vector_type<float, 2u> >, 1, 256>"),
    (True, "fp64_odd"): ("k_eo_hop<tip::CovOp<HIP_vector_type<double, 2u> >, 0, 5, 256, false>"
                         if os.environ.get("TIP_EO_WIDE") == "0"
                         else "k_eo_hop<tip::CovOp<HIP_vector_type<double, 2u> >, 0, 5, 512, false>"),
    (True, "fp32_odd"): ("k_eo_hop<tip::CovOp<HIP_vector_type<float, 2u> >, 0, 5, 256, false>"
                         if os.environ.get("TIP_EO_PAIR") == "0"
                         else "k_eo_hop_pair<tip::CovOp<HIP_vector_type<float, 2u> >, 0, 256>"),
    (False, "fp64"): "k_stencil_march4<HIP_vector_type<double, 2u>, 5, false>",
    (False, "fp32"): "k_stencil_march4<HIP_vector_type<float, 2u>, 5, false>",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_records():
    """The per-kernel records of the traffic file ([] when absent)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return []
    return t.get("records", [t] if "kernel" in t else [])


def measured_traffic(kernel_name):
    """HBM bytes per stencil launch of kernel_name from the committed rocprofv3
    counter runs, or None when there is no record of it or the kernel sources
    changed since it was taken."""
    src = kernel_source_hash()
    for t in traffic_records():
        if t.get("kernel") == kernel_name and t.get("source_sha256") == src:
            return t.get("traffic_bytes_per_launch")
    return None


def write_traffic(fetch_csv, write_csv, kernel_match, command):
    """Derive HBM bytes per stencil launch from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE, each taken with --copy-calibration) and store them with the
    hash of the kernel sources.  Each counter is scaled by what it reads for the
    plain 1 GiB device copy of the same run (read 2^30 bytes, written 2^30 bytes).
    Launches that moved under 1% of the largest one's bytes returned at once
    and are left out of the average."""
    import csv

    def per_launch(path, counter):
        copies, vals = [], []
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] != counter:
                    continue
                v = float(row["Counter_Value"])
                if "copyBuffer" in row["Kernel_Name"]:
                    copies.append(v)
                elif kernel_match in row["Kernel_Name"]:
                    vals.append(v)
        if not vals or not copies:
            raise SystemExit(f"{path}: no {counter} rows for {kernel_match!r} or for the calibration copy")
        # launches that returned at once (every rhs of the block already stopped)
        # are not stencil work: bench.py does not time them either
        vals = [v for v in vals if v > 0.01 * max(vals)]
        top = max(copies)
        calib = [c for c in copies if c > 0.9 * top]
        scale = float(1 << 30) / (1024.0 * sum(calib) / len(calib))
        return sum(vals) / len(vals), scale, len(vals)

    fk, fs, nf = per_launch(fetch_csv, "FETCH_SIZE")
    wk, ws, nw = per_launch(write_csv, "WRITE_SIZE")
    out = {"kernel": kernel_match, "source_sha256": kernel_source_hash(),
           "fetch_kib_per_launch": fk, "fetch_scale": fs, "write_kib_per_launch": wk, "write_scale": ws,
           "launches": [nf, nw], "traffic_bytes_per_launch": 1024.0 * (fk * fs + wk * ws), "command": command}
    # other kernels' records stay while they were taken on the same sources
    records = [t for t in traffic_records()
               if t.get("kernel") != kernel_match and t.get("source_sha256") == out["source_sha256"]] + [out]
    with open(TRAFFIC_FILE, "w") as f:
        json.dump({"records": records}, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


_ORACLE = {}


def _oracle_worker_init(seed, tol, barrier):
    """Worker of the all-cores oracle run: builds the same 32^4 operator
    (numpy on one thread), then waits for every other worker."""
    from threadpoolctl import threadpool_limits

    from oracle.hierperm import hier_perm
    from oracle.operators import Operator
    from paper_1302_4018_amd import inputs

    _ORACLE["limits"] = threadpool_limits(limits=1)
    _ORACLE["op"] = Operator(DIMS, 1, mass_field=inputs.mass_field(DIMS), links=inputs.haar_links(DIMS))
    _ORACLE["P"] = hier_perm(DIMS)
    _ORACLE["seed"], _ORACLE["tol"] = seed, tol
    barrier.wait()


def _oracle_worker_solve(k):
    """One complete oracle CG solve of right-hand side k; (start, end, iterations)."""
    from oracle.cg import cg_solve
    from oracle.mask import MASK_Z4
    from oracle.probing import rhs

    op = _ORACLE["op"]
    b = rhs(DIMS, 3, k // 3, k % 3, _ORACLE["seed"], MASK_Z4, _ORACLE["P"])
    t0 = time.time()
    _, it, _ = cg_solve(op.apply, b, _ORACLE["tol"], 10 * op.V * 3)
    return t0, time.time(), it


def host_cores():
    """CPUs this process may run on, capped at the 16-core share a one-GPU
    node gives each GPU."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(U, mf, seed, tol, n_rhs, all_cores=True):
    """The CPU oracle on a bounded sample: complete solves (textbook CG to the
    same true residual) of the first right-hand sides of this workload, on one
    host thread; then one solve per core on every core at once (one oracle
    process per core, each on one thread, distinct right-hand sides), timed
    from the moment all of them have their operator."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.cg import cg_solve
    from oracle.hierperm import hier_perm
    from oracle.mask import MASK_Z4
    from oracle.operators import Operator
    from oracle.probing import rhs

    with threadpool_limits(limits=1):
        op = Operator(DIMS, 1, mass_field=mf, links=U)
        P = hier_perm(DIMS)
        bs = [rhs(DIMS, 3, k // 3, k % 3, seed, MASK_Z4, P) for k in range(n_rhs)]
        iters = []
        q = 0.0 + 0.0j
        t0 = time.perf_counter()
        for k, b in enumerate(bs):
            x, it, _ = cg_solve(op.apply, b, tol, 10 * op.V * 3)
            iters.append(it)
            if k < 3:
                q += complex(np.vdot(b, x))           # q_0 = sum_c b_{0,c}^H x_{0,c}
        dt = time.perf_counter() - t0
    out = {"value": n_rhs / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": f"{n_rhs} complete oracle CG solves ({dt:.1f} s, {sum(iters) / len(iters):.1f} iterations each) "
                     f"of the first right-hand sides of the same 32^4 workload, one host thread",
           "nproc": os.cpu_count()}
    if n_rhs >= 3:
        out["_q0"] = q                                # probe 0 (three solves): the oracle's T_1
    if all_cores:
        n = host_cores()
        ctx = mp.get_context("spawn")                 # fresh processes: numpy only, nothing of the GPU
        barrier = ctx.Barrier(n)
        with ctx.Pool(n, initializer=_oracle_worker_init, initargs=(seed, tol, barrier)) as pool:
            res = pool.map(_oracle_worker_solve, range(n), chunksize=1)
        span = max(e for _, e, _ in res) - min(s0 for s0, _, _ in res)
        out["all_cores"] = {"value": n / span, "unit": "solves/s", "cores": n, "kind": "oracle",
                            "sample": f"{n} oracle processes on one thread each, one complete solve each (right-hand "
                                      f"sides 0..{n - 1}), all at once: {span:.1f} s from the first start to the "
                                      f"last end", "nproc": os.cpu_count()}
    return out


def per_estimate_errors(mixed, fp64, lam_lb, q0_oracle=None):
    """For every estimate T_k (s = 2^k) of the mixed-precision run: its relative
    difference from the FP64 run's, and the bound on its own error, (1/s)
    sum_{m<s,c} ||r||^2 / lambda_lb relative to T_k (its quadratures are the
    variational b^H x + x^H r, whose error is r^H A^-1 r; ||r||^2 = V res^2
    with the per-solve true residuals); at s = 1 both runs against the
    oracle's T_1 from its own solves of probe 0."""
    import numpy as np
    V = float(np.prod(DIMS))
    rows = []
    for k, (tm, tf) in enumerate(zip(mixed["est"], fp64["est"])):
        s = 1 << k
        bm = float(np.sum(V * mixed["residuals"][:s] ** 2) / lam_lb / s)
        row = {"s": s, "rel_diff_vs_fp64": float(abs(tm - tf) / abs(tf)), "bound_rel": bm / abs(tm)}
        if k == 0 and q0_oracle is not None:
            row["rel_err_vs_oracle_mixed"] = float(abs(tm - q0_oracle) / abs(q0_oracle))
            row["rel_err_vs_oracle_fp64"] = float(abs(tf - q0_oracle) / abs(q0_oracle))
        rows.append(row)
    return rows


def copy_calibration():
    """A plain 1 GiB device copy, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 1 << 27                                   # 2^27 doubles = 1 GiB
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {n * 8} bytes")


def bench_c4(args, emit=True):
    """The batch of 64 independent uneven 3-D tori (sides iid in [8, 48], scalar
    weighted Laplacian with m ~ U[0.02, 0.2], w ~ U[0.5, 1.5], Z2 mask, 16..256
    probes each) in one trace_inv_probe_batch call per step: every CG phase of
    every torus is one launch per group (real / complex probe classes), a
    chunk of iterations of the whole batch is one HIP graph.  FP32 CG with
    FP64 reliable updates (the headline of this line) and FP64 beside it.  The
    block size and work-item size come from tip_autotune_batch (cached).  The
    stencil roofline comes from one extra step with per-launch timing.
    Prints one JSON line (emit) or returns it."""
    import torch

    from paper_1302_4018_amd import autotune
    from paper_1302_4018_amd import binding as tip
    from paper_1302_4018_amd import inputs

    tori = inputs.uneven_tori()
    ops = []
    for i, t in enumerate(tori):
        w = torch.from_numpy(inputs.uneven_torus_couplings(t["dims"], i)).cuda()
        ops.append(tip.Operator(t["dims"], tip.KIND_SCALAR, mass=t["mass"], coupling=w))
    ns = [t["n_vectors"] for t in tori]
    total = sum(ns)
    if args.sequential:
        bench_c4_sequential(args, tip, ops, ns)
        return
    res = {}
    for name, prec in (("mixed", tip.PREC_MIXED), ("fp64", tip.PREC_FP64)):
        kw = {}
        if args.no_autotune:
            if args.rhs_block > 0:
                kw["rhs_block"] = args.rhs_block
            if args.item_sites > 0:
                kw["item_sites"] = args.item_sites
        else:
            t0 = time.perf_counter()
            kw = autotune.tuned_batch(ops, ns, args.tol, args.seed, mask=tip.MASK_Z2, precision=prec)
            log(f"[c4 {name}] tuning {kw} ({time.perf_counter() - t0:.1f} s)")
        for _ in range(args.warmup):
            tip.trace_inv_probe_batch(ops, ns, args.tol, args.seed, mask=tip.MASK_Z2, precision=prec, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        agg = {"iters": 0, "solves": 0, "relres": 0.0, "reused": 0, "ru": 0}
        for k in range(args.steps):
            out = tip.trace_inv_probe_batch(ops, ns, args.tol, args.seed, mask=tip.MASK_Z2, precision=prec, **kw)
            for _, st in out:
                agg["iters"] += st["total_iters"]
                agg["solves"] += st["solves"]
                agg["reused"] += st["reused"]
                agg["ru"] += st["reliable_updates"]
                agg["relres"] = max(agg["relres"], st["max_true_relres"])
            log(f"[c4 {name}] step {k}: {out[0][1]['seconds']:.3f} s")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tip.tip_set_profiling(True)
        st0 = tip.trace_inv_probe_batch(ops, ns, args.tol, args.seed, mask=tip.MASK_Z2, precision=prec, **kw)[0][1]
        tip.tip_set_profiling(False)
        res[name] = (total * args.steps / el, el, agg, st0, kw)
        log(f"[c4 {name}] {el / args.steps:.3f} s/step, {agg['iters'] / agg['solves']:.1f} it/solve, "
            f"{agg['ru'] / max(agg['solves'], 1):.2f} reliable updates/solve")
    value, el, agg, st0, kw = res["mixed"]

    def roof(st):
        sec, byt, n = st["stencil_seconds"], st["stencil_bytes"], st["stencil_launches"]
        ach = byt / sec / 1e9 if sec > 0 else 0.0
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "kb_stencil (batched generic site stencil, real and complex groups)",
                "alg_bytes_per_launch": byt / max(n, 1), "avg_launch_us": round(sec / max(n, 1) * 1e6, 2),
                "launches": n,
                "note": "algorithmic bytes of the live work items only (couplings once per site, p read and "
                        "w written per live rhs), counted on the device; from one extra step with eager launches"}
    out = {"metric": "probe quadratures/sec (batch of 64 uneven 3-D tori, rel.res 1e-10)", "value": round(value, 2),
           "unit": "quadratures/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(el / args.steps * 1e3, 2), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 CG + f64 reliable updates", "data": "synthetic",
           "config": {"workload": "64 independent 3-D tori, sides iid U{8..48}, scalar Laplacian m~U[0.02,0.2], "
                                  "w~U[0.5,1.5], Z2, 16..256 probes each, tol 1e-10",
                      "quadratures_per_step": total, "solves_per_step": agg["solves"] // args.steps,
                      "reused_conjugates_per_step": agg["reused"] // args.steps,
                      "iters_per_solve": round(agg["iters"] / agg["solves"], 2),
                      "max_true_relres": agg["relres"], "tuning": kw},
           "roofline": roof(st0), "cpu_baseline": None,
           "fp64": {"value": round(res["fp64"][0], 2), "ms_per_step": round(res["fp64"][1] / args.steps * 1e3, 2),
                    "iters_per_solve": round(res["fp64"][2]["iters"] / res["fp64"][2]["solves"], 2),
                    "tuning": res["fp64"][4], "roofline": roof(res["fp64"][3])}}
    if emit:
        print(json.dumps(out), flush=True)
    return out


def bench_c4_sequential(args, tip, ops, ns):
    """The same tori one after another on the calling thread (one
    trace_inv_probe per torus, mixed precision): the form a kernel trace can
    follow.  Prints one JSON line."""
    import torch
    handles = [tip.OpHandle(op) for op in ops]
    for _ in range(args.warmup):
        for h, n in zip(handles, ns):
            h.trace_inv_probe(n, args.tol, args.seed, mask=tip.MASK_Z2, precision=tip.PREC_MIXED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    quads = solves = 0
    for _ in range(args.steps):
        for h, n in zip(handles, ns):
            _, _, st = h.trace_inv_probe(n, args.tol, args.seed, mask=tip.MASK_Z2, precision=tip.PREC_MIXED)
            quads += n
            solves += st["solves"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for h in handles:
        h.close()
    print(json.dumps({"metric": "probe quadratures/sec, 64 uneven 3-D tori one after another (one thread)",
                      "value": round(quads / el, 1), "unit": "quadratures/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 2),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32 CG + f64 reliable updates", "data": "synthetic",
                      "config": {"workload": "64 independent 3-D tori, sides iid U{8..48}, sequential",
                                 "solves_per_s": round(solves / el, 1)}}), flush=True)


def bench_compare(args):
    """The comparison study of Sec. 5 on the GPU path: a 32^3 free torus with
    m = 0.05 (condition number about 240), whose Tr(A^-1) is known in closed
    form; the RMS over masks of the relative error of T_s at s = 2^k for the
    three probe kinds, up to s = 1024 (the 3-D completion points are 2, 16,
    128, 1024).  One JSON line; every solve is a FP64 CG to 1e-10 on the GPU."""
    import numpy as np
    import torch

    from paper_1302_4018_amd import binding as tip

    dims, m, n = [32, 32, 32], 0.05, 1024
    V = dims[0] * dims[1] * dims[2]
    k = np.arange(V)
    lam = m + sum(4.0 * np.sin(np.pi * ((k // st) % nn) / nn) ** 2
                  for nn, st in zip(dims, (1, dims[0], dims[0] * dims[1])))
    exact = float(np.sum(1.0 / lam))            # Fourier modes diagonalise the free torus (Sec. 5)
    gop = tip.Operator(dims, tip.KIND_SCALAR, mass=m)
    kinds = {"hierarchical": tip.PROBE_HIERARCHICAL, "natural": tip.PROBE_NATURAL, "random": tip.PROBE_RANDOM}
    table, solves = {}, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for name, probe in kinds.items():
        errs = []
        for seed in range(args.masks):
            est, _, st = tip.trace_inv_probe(gop, n, 1e-10, 1000 + seed, mask=tip.MASK_Z2, probe=probe)
            errs.append(np.abs(est.real - exact) / exact)
            solves += st["solves"]
        table[name] = [float(f"{v:.3e}") for v in np.sqrt(np.mean(np.array(errs) ** 2, axis=0))]
        log(f"[compare] {name}: {table[name]}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"metric": "relative error of T_s against the exact Tr(A^-1), RMS over masks (32^3 free torus, m=0.05)",
           "value": table["hierarchical"][-1], "unit": "relative error at s=1024", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": round(el * 1e3, 1), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "32^3 scalar Laplacian, m=0.05, Z2 masks, s = 1..1024", "masks": args.masks,
                      "exact_trace": exact, "s": [2 ** i for i in range(11)], "solves": solves,
                      "solves_per_s": round(solves / el, 1)},
           "errors": table}
    print(json.dumps(out), flush=True)


def bench_c2h(args):
    """The scalar weighted Laplacian at a size that does not fit in cache: a
    256^3 torus (V = 16.8M), w ~ U[0.5, 1.5] per forward edge, m = 0.05, Z2
    mask, one block of 32 probes solved to 1e-10 in FP64 (even-odd CG).  The
    roofline of its dominant kernel (the half-lattice S p stencil of the
    scalar operator) comes from hipEvent timing of every launch."""
    import numpy as np
    import torch

    from paper_1302_4018_amd import binding as tip
    from paper_1302_4018_amd import inputs

    dims, m, n = [256, 256, 256], 0.05, 32
    w = torch.from_numpy(inputs.couplings(dims)).cuda()
    op = tip.Operator(dims, tip.KIND_SCALAR, mass=m, coupling=w)
    with tip.OpHandle(op) as h:
        tip.tip_set_profiling(True)
        for _ in range(args.warmup):
            h.trace_inv_probe(n, args.tol, args.seed, mask=tip.MASK_Z2)
        tot = {"launches": 0, "seconds": 0.0, "bytes": 0.0, "iters": 0, "solves": 0, "relres": 0.0, "eo": 0}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            est, q, st = h.trace_inv_probe(n, args.tol, args.seed, mask=tip.MASK_Z2)
            for key, f in (("launches", "stencil_launches"), ("seconds", "stencil_seconds"),
                           ("bytes", "stencil_bytes"), ("iters", "total_iters"), ("solves", "solves")):
                tot[key] += st[f]
            tot["relres"] = max(tot["relres"], st["max_true_relres"])
            tot["eo"] = st["even_odd"]
            log(f"[c2h] step {k}: {st['seconds']:.3f} s, {st['total_iters'] / st['solves']:.1f} it/solve")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tip.tip_set_profiling(False)
    avg = tot["seconds"] / max(tot["launches"], 1)
    bpl = tot["bytes"] / max(tot["launches"], 1)
    ach = bpl / avg / 1e9 if avg > 0 else 0.0
    if not tot["eo"]:
        name = "k_stencil_march<ScalarOp<double>>"
    elif os.environ.get("TIP_EO_PAIR") == "0":
        name = "k_eo_hop<tip::ScalarOp<double>, 1, 5, 256, false>"
    else:
        name = "k_eo_hop_pair<tip::ScalarOp<double>, 1, 512>"
    out = {"metric": "scalar stencil HBM GB/s vs peak (3D 256^3 weighted Laplacian, rel.res 1e-10)",
           "value": round(ach, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(el / args.steps * 1e3, 2), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "3D 256^3 scalar weighted Laplacian, w~U[0.5,1.5], m=0.05, Z2, 32 probes, tol "
                                  f"{args.tol:g}", "solves_per_s": round(tot["solves"] / el, 2),
                      "iters_per_solve": round(tot["iters"] / max(tot["solves"], 1), 2),
                      "max_true_relres": tot["relres"], "even_odd": bool(tot["eo"])},
           "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": name,
                        "alg_bytes_per_launch": bpl, "avg_launch_us": round(avg * 1e6, 2),
                        "launches": tot["launches"]},
           "estimate": [float(np.real(est[-1]))]}
    print(json.dumps(out), flush=True)


def _configs_oracle_sample(cfg, n_probe, seed):
    """The oracle on the first n_probe probes of a small configuration, on
    this thread: (seconds, solves, estimates)."""
    import numpy as np

    from oracle.estimator import trace_inv_probe as oracle_trace

    t = time.perf_counter()
    est, _, st = oracle_trace(cfg["oracle_op"](), n_probe, cfg["tol"], seed, cfg["mask_o"])
    return time.perf_counter() - t, len(st["iters"]), np.asarray(est)



def bench_configs(args):
    """The three small configurations beside the 32^4 one: C1 (2-D 16^2 free
    scalar Laplacian, m = 0.1, all 256 probes, tol 1e-12: the estimate is then
    Tr(A^-1) itself), C2 (3-D 32^3 weighted Laplacian, w ~ U[0.5, 1.5],
    m = 0.05, 512 probes, tol 1e-10), C3 (4-D 16^4 covariant Laplacian, Haar
    U(3) links, m = 0.1, Z4, 1024 probes x 3 components, tol 1e-10).  Each
    runs on the GPU (one warm-up call, then K timed calls with the operator
    resident) and in the oracle on one host thread (C1 whole, C2 and C3 on a
    sample of their first probes), and the GPU's estimates at the sample's
    checkpoints are compared with the oracle's.  These working sets sit in
    L2 / MALL, so no HBM roofline is quoted for them.  Prints one JSON line."""
    import numpy as np
    import torch

    from oracle.mask import MASK_Z2 as OZ2, MASK_Z4 as OZ4
    from oracle.operators import Operator as OOp
    from paper_1302_4018_amd import binding as tip
    from paper_1302_4018_amd import inputs

    d1, d2, d3 = [16, 16], [32, 32, 32], [16, 16, 16, 16]
    w2 = inputs.couplings(d2, seed=1)
    U3 = inputs.haar_links(d3, seed=3)
    cfgs = [
        {"name": "C1", "workload": "2D 16^2 scalar Laplacian, m=0.1, Z2, 256 probes (all sites), tol 1e-12",
         "op": lambda: tip.Operator(d1, tip.KIND_SCALAR, mass=0.1), "oracle_op": lambda: OOp(d1, 0, mass=0.1),
         "n": 256, "tol": 1e-12, "mask": tip.MASK_Z2, "mask_o": OZ2, "sample": 256},
        {"name": "C2", "workload": "3D 32^3 weighted Laplacian, w~U[0.5,1.5], m=0.05, Z2, 512 probes, tol 1e-10",
         "op": lambda: tip.Operator(d2, tip.KIND_SCALAR, mass=0.05, coupling=torch.from_numpy(w2).cuda()),
         "oracle_op": lambda: OOp(d2, 0, mass=0.05, coupling=w2),
         "n": 512, "tol": 1e-10, "mask": tip.MASK_Z2, "mask_o": OZ2, "sample": 32},
        {"name": "C3", "workload": "4D 16^4 covariant Laplacian x3, Haar U(3) links, m=0.1, Z4, 1024 probes x 3, "
                                   "tol 1e-10",
         "op": lambda: tip.Operator(d3, tip.KIND_COVARIANT, mass=0.1, links=torch.from_numpy(U3).cuda()),
         "oracle_op": lambda: OOp(d3, 1, mass=0.1, links=U3),
         "n": 1024, "tol": 1e-10, "mask": tip.MASK_Z4, "mask_o": OZ4, "sample": 2},
    ]
    rows = []
    for c in cfgs:
        with tip.OpHandle(c["op"]()) as h:
            for _ in range(max(args.warmup, 1)):
                h.trace_inv_probe(c["n"], c["tol"], args.seed, mask=c["mask"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solves = iters = 0
            relres = 0.0
            for _ in range(args.steps):
                est, _, st = h.trace_inv_probe(c["n"], c["tol"], args.seed, mask=c["mask"])
                solves += st["solves"]
                iters += st["total_iters"]
                relres = max(relres, st["max_true_relres"])
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        sec, n_o, est_o = _configs_oracle_sample(c, c["sample"], args.seed)
        k = len(est_o)
        parity = float(np.max(np.abs(est[:k] - est_o) / np.abs(est_o)))
        log(f"[{c['name']}] GPU {solves / el:.1f} solves/s, oracle {n_o / sec:.3f} solves/s ({c['sample']} probes, "
            f"{sec:.1f} s), max rel. diff of T_s up to s = {c['sample']}: {parity:.2e}")
        rows.append({"config": c["name"], "workload": c["workload"],
                     "gpu": {"solves_per_s": round(solves / el, 2), "ms_per_call": round(el / args.steps * 1e3, 2),
                             "iters_per_solve": round(iters / max(solves, 1), 2), "max_true_relres": relres,
                             "even_odd": bool(st["even_odd"]), "estimate": float(np.real(est[-1]))},
                     "oracle": {"solves_per_s": round(n_o / sec, 4), "cores": 1, "kind": "oracle",
                                "sample": f"probes 0..{c['sample'] - 1} ({n_o} complete CG solves, {sec:.1f} s), "
                                          "one host thread"},
                     "parity_max_rel_diff_T_s": parity})
    out = {"metric": "probing-vector solves/sec on the small configurations (GPU and oracle)",
           "value": None, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "data": "synthetic", "dtype": "f64", "configs": rows}
    print(json.dumps(out), flush=True)


def free_spectrum(dims, m):
    """Eigenvalues m + sum_mu 4 sin^2(pi k_mu / n_mu) of the free shifted
    Laplacian (its Fourier modes diagonalise it), one per site."""
    import numpy as np
    grids = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    return (m + sum(4.0 * np.sin(np.pi * k / n) ** 2 for k, n in zip(grids, dims))).ravel()


def bench_study(args):
    """The experiments of Sec. 5 on the GPU path, every solve a FP64 CG to 1e-10.

    A (Sec. 5.1): 64^3 free torus at condition number 100, no mask; the
      hierarchy stopped after 1..5 bit-levels against the full one (6 levels).
    B (Sec. 5.2): the three lattices 64^3, 32^4 and 64 x 128^2 at condition
      numbers 1e2, 1e4 and 1e6; hierarchical, Fourier-grouped, natural-order
      Hadamard and random Z2 probes, RMS over Z2 masks of the relative error.
    C (Sec. 5.2, variance over 100 masks): 16^4 at condition number 100; the
      sample variance over masks of the hierarchical T_s against the exact
      variance of plain Z2 Monte Carlo with s vectors, 2 (sum 1/lam^2 -
      (sum 1/lam)^2 / V) / s, and their ratio (the variance reduction at equal
      work).
    The free tori have Tr(A^-1) = sum_k 1/lam(k) in closed form."""
    import numpy as np
    import torch

    from paper_1302_4018_amd import binding as tip

    def exact(dims, m):
        lam = free_spectrum(dims, m)
        return float(np.sum(1.0 / lam)), float(np.sum(lam ** -2.0))

    def mass_for(dims, kappa):                 # lam_max = m + 4 d, lam_min = m
        return 4.0 * len(dims) / (kappa - 1.0)

    out = {"metric": "relative error of T_s against the exact Tr(A^-1) (Sec. 5 study)", "n_gpus": 1,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "unit": "relative error", "steps": 1, "warmup": 0}
    solves = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    parts = set(args.study.split(","))

    if "A" in parts:
        dims, kappa, n = [64, 64, 64], 100.0, 4096
        m = mass_for(dims, kappa)
        tr, _ = exact(dims, m)
        table = {}
        with tip.OpHandle(tip.Operator(dims, tip.KIND_SCALAR, mass=m)) as h:
            for lev in (1, 2, 3, 4, 5, 6):
                est, _, st = h.trace_inv_probe(n, args.tol, 1, mask=tip.MASK_NONE, probe=tip.PROBE_STOPPED,
                                               stop_levels=lev)
                solves += st["solves"]
                table[f"levels={lev}"] = [float(f"{v:.3e}") for v in np.abs(est.real - tr) / tr]
                log(f"[study A] stopped at {lev} levels: {table[f'levels={lev}']}")
        out["A_stopped_levels"] = {"lattice": dims, "kappa": kappa, "mass": m, "mask": "none", "exact_trace": tr,
                                   "s": [2 ** i for i in range(13)], "rel_error": table}

    if "B" in parts:
        kinds = {"hierarchical": tip.PROBE_HIERARCHICAL, "fourier_grouped": tip.PROBE_FOURIER,
                 "natural": tip.PROBE_NATURAL, "random_z2": tip.PROBE_RANDOM}
        res = {}
        for dims, kappa, n in (([64, 64, 64], 1e2, 4096), ([32, 32, 32, 32], 1e4, 1024),
                               ([64, 128, 128], 1e6, 256)):
            m = mass_for(dims, kappa)
            tr, _ = exact(dims, m)
            name = "x".join(map(str, dims))
            # FP64 CG reaches a true relative residual of about eps * kappa, so at
            # kappa = 1e6 the solves stop at 1e-8; the quadrature error is then
            # <= kappa tol^2 = 1e-10, far below the estimator errors compared here
            tol_b = max(args.tol, 1e-8) if kappa > 1e5 else args.tol
            rows = {}
            with tip.OpHandle(tip.Operator(dims, tip.KIND_SCALAR, mass=m)) as h:
                for kname, probe in kinds.items():
                    errs = []
                    for seed in range(args.masks):
                        est, _, st = h.trace_inv_probe(n, tol_b, 1000 + seed, mask=tip.MASK_Z2, probe=probe,
                                                       max_iter=200000)
                        solves += st["solves"]
                        errs.append(np.abs(est.real - tr) / tr)
                    rows[kname] = [float(f"{v:.3e}") for v in np.sqrt(np.mean(np.array(errs) ** 2, axis=0))]
                    log(f"[study B] {name} kappa {kappa:g} {kname}: {rows[kname]}")
            res[name] = {"kappa": kappa, "mass": m, "tol": tol_b, "exact_trace": tr,
                         "s": [2 ** i for i in range(len(rows["natural"]))], "rms_rel_error": rows}
        out["B_vs_monte_carlo"] = {"masks": args.masks, "lattices": res}

    if "C" in parts:
        dims, kappa, n, masks = [16, 16, 16, 16], 100.0, 1024, args.variance_masks
        m = mass_for(dims, kappa)
        tr, tr2 = exact(dims, m)
        V = int(np.prod(dims))
        var_q = 2.0 * (tr2 - tr * tr / V)                  # one Z2 quadrature: 2 sum_{x != y} G(x - y)^2
        ests = []
        with tip.OpHandle(tip.Operator(dims, tip.KIND_SCALAR, mass=m)) as h:
            for seed in range(masks):
                est, _, st = h.trace_inv_probe(n, args.tol, 5000 + seed, mask=tip.MASK_Z2)
                solves += st["solves"]
                ests.append(est.real)
        ests = np.array(ests)
        s = np.array([2 ** i for i in range(ests.shape[1])], dtype=float)
        var_hp = np.var(ests, axis=0, ddof=1)
        var_mc = var_q / s
        out["C_variance"] = {"lattice": dims, "kappa": kappa, "mass": m, "masks": masks, "exact_trace": tr,
                             "s": s.astype(int).tolist(),
                             "mean_rel_error": [float(f"{v:.3e}") for v in np.abs(ests.mean(axis=0) - tr) / tr],
                             "var_hierarchical": [float(f"{v:.4e}") for v in var_hp],
                             "var_monte_carlo_exact": [float(f"{v:.4e}") for v in var_mc],
                             "reduction": [float(f"{v:.4g}") for v in var_mc / np.maximum(var_hp, 1e-300)]}
        log(f"[study C] variance reduction at s = 2^k: {out['C_variance']['reduction']}")

    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["ms_per_step"] = round(el * 1e3, 1)
    out["config"] = {"workload": "Sec. 5 study on free shifted Laplacians (parts " + ",".join(sorted(parts)) + ")",
                     "solves": solves, "solves_per_s": round(solves / el, 1), "tol": args.tol}
    first = out.get("C_variance", {}).get("reduction") or [None]
    out["value"] = first[-1]
    out["unit"] = "variance reduction over Z2 Monte Carlo at s=1024 (16^4, 100 masks)" if first[-1] else "see parts"
    out["higher_is_better"] = True
    print(json.dumps(out), flush=True)


def practical_ceiling(tip):
    """The HBM rate hand-written streaming kernels reach on this GPU (tip_stream_ceiling:
    4 GiB, 8192 workgroups of 256 threads, 16-byte accesses), read only and three reads
    per write, in GB/s; measured outside the timed steps."""
    out = {"unit": "GB/s", "bytes": 4 << 30}
    for kind, key in ((0, "read_only"), (2, "three_reads_one_write")):
        sec, byt = tip.tip_stream_ceiling(kind, 4 << 30, 10, 8192)
        out[key] = round(byt / sec / 1e9, 1)
    return out


def timed_gradient(handle, args, n_rhs, forward):
    """The same probing run with the gradient of the last estimate with respect
    to the mass field and the couplings (trace_inv_probe_grad, FP64): W warmup
    and K timed calls, reported as solves/s beside the forward-only rate."""
    import numpy as np
    import torch

    kw = dict(rhs_block=args.rhs_block)
    for w in range(args.warmup):
        handle.trace_inv_probe_grad(args.n_vectors, args.tol, args.seed, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        est, _, gm, gw, st = handle.trace_inv_probe_grad(args.n_vectors, args.tol, args.seed, **kw)
        log(f"[gradient] step {k}: {st['seconds']:.3f} s, {st['solves']} solves")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = n_rhs * args.steps / elapsed
    return {"value": round(value, 2), "unit": "solves/s", "ms_per_step": round(elapsed / args.steps * 1e3, 2),
            "vs_forward_fp64": round(value / forward["value"], 3), "dtype": "f64",
            "outputs": "estimates, dT/dm [V] and dT/dw [ndim][V] of the last estimate",
            "max_rel_diff_estimates_vs_forward": float(np.max(np.abs(est - forward["est"]) / np.abs(forward["est"]))),
            "grad_mass_sum": float(gm.sum()), "grad_coupling_sum": float(gw.sum())}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-vectors", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--rhs-block", type=int, default=0)
    ap.add_argument("--item-sites", type=int, default=0,
                    help="c4 with --no-autotune: sites per work item of the batched solver (0 = library default)")
    ap.add_argument("--seed", type=int, default=4018)
    ap.add_argument("--cpu-solves", type=int, default=3, help="right-hand sides the CPU oracle solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-one-core", action="store_true", help="time the oracle on one host thread only")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch of 64 uneven 3-D tori that the default line reports under batch_c4")
    ap.add_argument("--no-gradient", action="store_true",
                    help="skip the leg that times the estimate together with dT/dm and dT/dw")
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both",
                    help="FP64 is the headline value; 'both' adds the mixed-precision solver beside it")
    ap.add_argument("--reliable-delta", type=float, default=0.0)
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the stencil's measured HBM bytes per launch from two rocprofv3 --pmc "
                         "counter_collection.csv files, then exit (no GPU work)")
    ap.add_argument("--traffic-command", default="", help="command recorded with --traffic-from")
    ap.add_argument("--traffic-kernel", choices=["fp64", "fp32", "fp64_odd", "fp32_odd"], default="fp64",
                    help="--traffic-from: the FP64 or the single-precision dominant kernel of the 32^4 workload")
    ap.add_argument("--workload", choices=["c5", "c4", "c2h", "configs", "compare", "study"], default="c5",
                    help="c5: the 32^4 covariant probing run (default); c4: the batch of 64 uneven 3-D tori; "
                         "c2h: the scalar stencil's HBM rate on a 256^3 torus; configs: C1, C2, C3 on the GPU "
                         "and in the oracle; "
                         "compare: hierarchical vs natural-order Hadamard vs Monte-Carlo probes on a 32^3 torus "
                         "with a closed-form trace; study: the experiments of Sec. 5 (stopped levels, three "
                         "lattices and condition numbers, variance over 100 masks)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="c4: the library's default block and work-item sizes instead of tip_autotune_batch")
    ap.add_argument("--masks", type=int, default=4, help="compare / study B: masks averaged per probe kind")
    ap.add_argument("--sequential", action="store_true",
                    help="c4: solve the tori one after another on one thread instead of the batch call")
    ap.add_argument("--study", default="A,B,C", help="study: parts to run (A stopped levels, B lattices x "
                    "condition numbers, C variance over masks)")
    ap.add_argument("--variance-masks", type=int, default=100, help="study C: masks")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(args.traffic_from[0], args.traffic_from[1], STENCIL[(True, args.traffic_kernel)],
                      args.traffic_command)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "sharding the probe indices over GPUs with one final all-reduce is designed, not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1302_4018_amd import binding as tip
    from paper_1302_4018_amd import inputs

    if args.copy_calibration:
        copy_calibration()

    if args.workload == "c4":
        bench_c4(args)
        return
    if args.workload == "compare":
        bench_compare(args)
        return
    if args.workload == "study":
        bench_study(args)
        return
    if args.workload == "c2h":
        bench_c2h(args)
        return
    if args.workload == "configs":
        bench_configs(args)
        return

    t = time.perf_counter()
    U = inputs.haar_links(DIMS)
    mf = inputs.mass_field(DIMS)
    log(f"inputs generated in {time.perf_counter() - t:.1f} s")
    dev_U = torch.from_numpy(U).cuda()
    dev_mf = torch.from_numpy(mf).cuda()
    op = tip.Operator(DIMS, tip.KIND_COVARIANT, mass_field=dev_mf, links=dev_U)
    torch.cuda.synchronize()
    t = time.perf_counter()
    handle = tip.OpHandle(op)
    torch.cuda.synchronize()
    repack_s = time.perf_counter() - t
    log(f"operator handle (link repack) {repack_s * 1e3:.1f} ms")

    n_rhs = args.n_vectors * 3

    def timed(precision):
        """W warmup calls, then K timed calls of the whole path at one precision
        (as a user runs it: chunks of iterations replayed as HIP graphs), then
        one more call with every launch timed by hipEvents (eager launches) for
        the roofline of the dominant kernel."""
        tip.tip_set_profiling(False)
        kw = dict(rhs_block=args.rhs_block, precision=precision, reliable_delta=args.reliable_delta)
        for w in range(args.warmup):
            est, q, st = handle.trace_inv_probe(args.n_vectors, args.tol, args.seed, **kw)
            log(f"[{precision}] warmup {w}: {st['seconds']:.3f} s, {st['total_iters'] / st['solves']:.2f} it/solve")
        tot = {"launches": 0, "seconds": 0.0, "bytes": 0.0, "iters": 0, "solves": 0, "relres": 0.0, "ru": 0,
               "bound": 0.0, "mv": 0, "mv_seconds": 0.0, "mv_bytes": 0.0, "eo": False}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            est, q, st = handle.trace_inv_probe(args.n_vectors, args.tol, args.seed, **kw)
            tot["iters"] += st["total_iters"]
            tot["solves"] += st["solves"]
            tot["ru"] += st["reliable_updates"]
            tot["relres"] = max(tot["relres"], st["max_true_relres"])
            tot["bound"] = max(tot["bound"], st["max_quad_err_bound"])
            tot["eo"] = bool(st["even_odd"])
            log(f"[{precision}] step {k}: {st['seconds']:.3f} s, {st['solves']} solves, "
                f"max rel.res {st['max_true_relres']:.2e}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        tip.tip_set_profiling(True)
        _, _, sp = handle.trace_inv_probe(args.n_vectors, args.tol, args.seed, **kw)
        tip.tip_set_profiling(False)
        tot["launches"] = sp["stencil_launches"]
        tot["seconds"] = sp["stencil_seconds"]
        tot["bytes"] = sp["stencil_bytes"]
        tot["mv"] = sp["matvecs"]
        tot["mv_seconds"] = sp["matvec_seconds"]
        tot["mv_bytes"] = sp["matvec_bytes"]
        avg_launch_s = tot["seconds"] / max(tot["launches"], 1)
        bytes_per_launch = tot["bytes"] / max(tot["launches"], 1)
        achieved = bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
        name = STENCIL[(tot["eo"], "fp64" if precision == tip.PREC_FP64 else "fp32")]
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name),
                "kernel": name, "alg_bytes_per_launch": bytes_per_launch,
                "avg_launch_us": round(avg_launch_s * 1e6, 2), "launches": tot["launches"]}
        if tot["mv"] and tot["mv_seconds"] > 0:
            # the whole operator application (both half-lattice kernels with the reduction)
            roof["operator"] = {"applications": tot["mv"], "avg_us": round(tot["mv_seconds"] / tot["mv"] * 1e6, 2),
                                "alg_bytes": tot["mv_bytes"] / tot["mv"],
                                "achieved": round(tot["mv_bytes"] / tot["mv_seconds"] / 1e9, 1)}
            if tot["eo"] and tot["mv"] == tot["launches"]:
                # the other half-lattice kernel of each application (t_o = D_o^-1 H_oe p_e),
                # timed between the same events: the operator minus the dominant kernel
                odd_s = (tot["mv_seconds"] - tot["seconds"]) / tot["mv"]
                odd_b = (tot["mv_bytes"] - tot["bytes"]) / tot["mv"]
                odd_name = STENCIL[(True, ("fp64" if precision == tip.PREC_FP64 else "fp32") + "_odd")]
                roof["odd_hop"] = {"kernel": odd_name, "avg_launch_us": round(odd_s * 1e6, 2),
                                   "alg_bytes_per_launch": odd_b, "achieved": round(odd_b / odd_s / 1e9, 1),
                                   "frac": round(odd_b / odd_s / 1e9 / HBM_PEAK_GBS, 4),
                                   "traffic": measured_traffic(odd_name)}
        return {"value": n_rhs * args.steps / elapsed, "elapsed": elapsed, "roofline": roof, "est": est, "eo": tot["eo"],
                "q": q, "residuals": st["residuals"],
                "iters_per_solve": tot["iters"] / max(tot["solves"], 1), "max_true_relres": tot["relres"],
                "reliable_updates_per_step": tot["ru"] / args.steps, "max_quad_err_bound": tot["bound"]}

    precisions = {"fp64": [tip.PREC_FP64], "mixed": [tip.PREC_MIXED],
                  "both": [tip.PREC_FP64, tip.PREC_MIXED]}[args.precision]
    res = {pr: timed(pr) for pr in precisions}
    grad = None if args.no_gradient else timed_gradient(handle, args, n_rhs, res[precisions[0]])
    handle.close()
    batch = None
    if not args.no_batch:
        # the batched solver on the 64 uneven 3-D tori, beside the 32^4 line
        c4 = bench_c4(args, emit=False)
        batch = {"metric": c4["metric"], "value": c4["value"], "unit": c4["unit"], "ms_per_step": c4["ms_per_step"],
                 "dtype": c4["dtype"], "workload": c4["config"]["workload"], "tuning": c4["config"]["tuning"],
                 "iters_per_solve": c4["config"]["iters_per_solve"], "max_true_relres": c4["config"]["max_true_relres"],
                 "fp64": {"value": c4["fp64"]["value"], "ms_per_step": c4["fp64"]["ms_per_step"]},
                 "roofline": c4["roofline"]}
    ceiling = practical_ceiling(tip)
    log(f"practical HBM ceiling: {ceiling}")
    for r in res.values():
        # the dominant kernel reads about four bytes for each one it writes
        r["roofline"]["practical_ceiling"] = ceiling
        r["roofline"]["frac_of_practical"] = round(r["roofline"]["achieved"] / ceiling["three_reads_one_write"], 4)
    main_pr = precisions[0]
    main = res[main_pr]
    value = main["value"]
    elapsed = main["elapsed"]
    iters_per_solve = main["iters_per_solve"]
    roofline = main["roofline"]
    est = main["est"]
    log(f"T_k estimates: {[round(float(v.real), 6) for v in est]}")
    mixed = None
    if tip.PREC_MIXED in res and main_pr != tip.PREC_MIXED:
        m = res[tip.PREC_MIXED]
        mixed = {"value": round(m["value"], 2), "unit": "solves/s", "ms_per_step": round(m["elapsed"] / args.steps * 1e3, 2),
                 "speedup_vs_fp64": round(m["value"] / value, 3), "dtype": "f32 CG + f64 reliable updates",
                 "iters_per_solve": round(m["iters_per_solve"], 2),
                 "reliable_updates_per_solve": round(m["reliable_updates_per_step"] / n_rhs, 2),
                 "max_true_relres": m["max_true_relres"], "max_quad_err_bound": m["max_quad_err_bound"],
                 "max_rel_diff_estimates_vs_fp64": float(np.max(np.abs(m["est"] - est) / np.abs(est))),
                 "roofline": m["roofline"]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(U, mf, args.seed, args.tol, args.cpu_solves, all_cores=not args.cpu_one_core)
    q0_oracle = cpu.pop("_q0", None) if cpu else None
    if mixed is not None:
        mixed["per_estimate"] = per_estimate_errors(res[tip.PREC_MIXED], main, float(np.min(mf)), q0_oracle)

    out = {"metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if main_pr == tip.PREC_FP64 else "f32 CG + f64 reliable updates", "data": "synthetic",
           "config": {"workload": "4D 32^4 covariant Laplacian x3 (Haar U(3) links, m(x)=0.1+0.02clip(xi)), "
                                  f"{args.n_vectors} hierarchical probes x 3 = {n_rhs} CG solves, tol {args.tol:g}",
                      "lattice": DIMS, "n_vectors": args.n_vectors, "rhs_per_step": n_rhs, "tol": args.tol,
                      "spatial_probes_per_s": round(value / 3, 2),
                      "mask": "Z4", "iters_per_solve": round(iters_per_solve, 2),
                      "solver": "CG on the even-odd reduced system" if main["eo"] else "CG",
                      "max_true_relres": main["max_true_relres"], "repack_ms": round(repack_s * 1e3, 2)},
           "roofline": roofline, "cpu_baseline": cpu, "mixed_precision": mixed, "gradient": grad,
           "batch_c4": batch}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
