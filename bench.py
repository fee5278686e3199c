#!/usr/bin/env python3
"""Benchmark of the red-black domain-wall path on one MI355X.

Default workload (FP64, the 16^3 x 32 lattice with Ls = 16, M5 = 1.8,
mf = 0.01, links exp(0.2 i H), Gaussian source): one *step* is a full
red-black solve of D_DW psi = eta to a relative residual of 1e-10 -- the
Schur source, CG on M_pc^dag M_pc, and the odd-site reconstruction -- with
the source already resident in HBM.

Printed (one JSON line): 5D site-updates/s counted as in the paper (one CG
iteration = two full matrix multiplies, M_pc = one, i.e. 2 * V5
site-updates per iteration), the roofline of the hopping kernels measured
with HIP events over the timed region, and the FP64 oracle timed on the
host on a bounded sample.

Other workloads (``--workload``): ``batched`` (40 complex64 vectors,
order-32 Chebyshev filter over [0.05, 60] and FP64-accumulated
Gram-Schmidt), ``mixed`` (24^3 x 48, Ls = 24, mf = 0.00078: Chebyshev setup
of 24 vectors + 2 CG solves, FP64 against FP16+scale storage), ``force``
(8^3 x 16, Ls = 12: dS/dU of the pseudofermion action), ``coarse``
(coarse-space transfer), ``krylov`` (the Krylov table's solvers) and
``hdcr`` (the two-level HDCR solver against the red-black CG solve).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MdagM 5D site-updates/s + HBM GB/s; Chebyshev setup vecs/s, FP64 vs mixed/batched"
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "rb_solve": dict(dims=(16, 16, 16, 32), Ls=16, M5=1.8, mf=0.01, eps=0.2),
    "batched": dict(dims=(16, 16, 16, 32), Ls=16, M5=1.8, mf=0.01, eps=0.2, nvec=40, order=32, lo=0.05, hi=60.0),
    "mixed": dict(dims=(24, 24, 24, 48), Ls=24, M5=1.8, mf=0.00078, eps=0.15, nvec=24, order=32, lo=0.05, hi=60.0),
    "force": dict(dims=(8, 8, 8, 16), Ls=12, M5=1.8, mf=0.01, eps=0.2),
    "copy": dict(bytes=4 << 30),
    # M_pc^dag M_pc alone on the 16^3x32 (Ls 16, links exp(0.2iH)) or 24^3x48 (Ls 24, exp(0.15iH)) lattice
    "operator": dict(lattices={"16x16x16x32": ((16, 16, 16, 32), 16, 0.2), "24x24x24x48": ((24, 24, 24, 48), 24, 0.15)},
                     M5=1.8, mf=0.01),
    "krylov": dict(dims=(16, 16, 16, 32), Ls=16, M5=1.8, mf=0.01, eps=0.2, tol=1e-10),
    # Algorithm A: 4x2x4x2 blocks, 40 basis vectors; Algorithm B: 2^4 blocks, 32 (both chirality-split)
    "coarse": dict(dims=(16, 16, 16, 32), Ls=16, M5=1.8, mf=0.01, eps=0.2, algos={"A": ((4, 2, 4, 2), 20), "B": ((2, 2, 2, 2), 16)}),
    # Algorithm B at the HDCR tables' light mass: setup filter (m, lo, hi), smoother (lo, hi, order);
    # Algorithm A (4x2x4x2 blocks, 20 + 20 chiral vectors) as a second leg
    "hdcr": dict(dims=(16, 16, 16, 32), Ls=16, M5=1.8, mf=0.001, eps=0.2, tol=1e-10, block=(2, 2, 2, 2), nraw=16,
                 filter=(300, 0.05, 70.0), smoother=(0.5, 70.0, 16), coarse_tol=0.02, nkrylov=8,
                 algorithm_a=dict(block=(4, 2, 4, 2), nraw=20)),
}

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hop_traffic.json")
HOP_SOURCE = os.path.join(ROOT, "paper_2103_05034_amd", "csrc", "hop.hip")

SPINOR_BYTES = {0: 192, 1: 96, 2: 52}
LINK_BYTES = {0: 144, 1: 72, 2: 72}


def hop_bytes_per_site(prec, Ls, nrhs=1):
    """Algorithmic HBM bytes per output even 5D site and rhs of the two hop passes of M_pc.

    pass 1 (t = M5D^-1 D_hop in): read in, write t      -> 2 S + 8 L / (Ls nrhs)
    pass 2 (out = M5D in - D_hop t / 4): read t, in, write out -> 3 S + 8 L / (Ls nrhs)
    """
    S, Lb = SPINOR_BYTES[prec], LINK_BYTES[prec]
    link = 8.0 * Lb / (Ls * nrhs)
    return 2 * S + link, 3 * S + link


# hop launches of one FP64 CG iteration, as (kernel-name prefix, algorithmic spinor reads + writes):
# M_pc p (pass 1: 2 S, pass 2 with p.Ap partials: 3 S), then M_pc^dag u with the residual update
# fused into its second pass (reads t, u, r and writes r: 4 S); each pass also reads 8 L / Ls of links
CG_ITERATION_HOPS = (
    ("void dwf::hop_kernel<0, 0, 0, false, 1,", 2),
    ("void dwf::hop_kernel<0, 0, 0, false, 2,", 3),
    ("void dwf::hop_kernel<0, 0, 0, true, 1,", 2),
    ("void dwf::hop_kernel<0, 0, 0, true, 4,", 4),
)


# kernels whose counters `--traffic` summarises, per workload: the four hop launches of a CG
# iteration, and the four passes of a Chebyshev step of the 40-rhs FP32 filter (M_pc: M5D^-1 and
# M5D epilogues; M_pc^dag: M5D^-dag, then the recurrence fused into the last pass)
TRAFFIC_KERNELS = {
    "rb_solve": [p for p, _ in CG_ITERATION_HOPS],
    "batched": [
        "void dwf::hop_kernel<1, 1, 1, false, 1,",
        "void dwf::hop_kernel<1, 1, 1, false, 2,",
        "void dwf::hop_kernel<1, 1, 1, true, 1,",
        "void dwf::hop_kernel<1, 1, 1, true, 3,",
    ],
}
# dispatches of each kind taken (the last ones: the timed work, after any autotuning)
TRAFFIC_LAST = {"rb_solve": None, "batched": 24}


def cg_hop_bytes_per_launch(V5h, Ls):
    """Algorithmic HBM bytes per hop launch, averaged over the four launches of a CG iteration."""
    S, Lb = SPINOR_BYTES[0], LINK_BYTES[0]
    per_site = sum(n for _, n in CG_ITERATION_HOPS) / len(CG_ITERATION_HOPS) * S + 8.0 * Lb / Ls
    return V5h * per_site


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, prefixes=None, last=None):
    """HBM bytes per hop launch of a CG iteration from four rocprofv3 --pmc runs (FETCH_SIZE and
    WRITE_SIZE of the rb_solve bench, and of the copy workload).  Each counter is scaled by the
    factor that maps its reading on the copy kernel (copy_bytes read, copy_bytes written) onto
    the known size; the result is the mean over the four launch kinds of a CG iteration (or over
    the kernels named by `prefixes`), each over its last `last` dispatches if given."""
    import csv
    import glob
    from collections import defaultdict

    def per_dispatch(d):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += list(csv.DictReader(open(f)))
        acc = defaultdict(float)
        names = {}
        for r in rows:
            acc[int(r["Dispatch_Id"])] += float(r["Counter_Value"])
            names[int(r["Dispatch_Id"])] = r["Kernel_Name"]
        return [(names[k], acc[k] * 1024.0) for k in sorted(acc)]  # counters are KiB per dispatch

    def copy_kib(d):
        return max(v for _, v in per_dispatch(d))  # the 4 GiB copy dominates every other dispatch

    f_scale = copy_bytes / copy_kib(copy_fetch_dir)
    w_scale = copy_bytes / copy_kib(copy_write_dir)
    fetch, write = per_dispatch(fetch_dir), per_dispatch(write_dir)
    kinds = {}
    for prefix in prefixes or [p for p, _ in CG_ITERATION_HOPS]:
        fv = [v for n, v in fetch if n.startswith(prefix)][-(last or 0):]
        wv = [v for n, v in write if n.startswith(prefix)][-(last or 0):]
        if not fv or not wv:
            raise SystemExit(f"no dispatch of {prefix!r} in the counter runs")
        kinds[prefix] = {
            "fetch_bytes": f_scale * sum(fv) / len(fv),
            "write_bytes": w_scale * sum(wv) / len(wv),
            "dispatches": len(fv),
        }
    per_launch = sum(k["fetch_bytes"] + k["write_bytes"] for k in kinds.values()) / len(kinds)
    return {"fetch_scale": f_scale, "write_scale": w_scale, "kinds": kinds, "bytes_per_launch": per_launch}


HOP_SAMPLE = 5  # hop launches per timed one in the timed solves


def rb_site_updates(V5, iterations):
    """5D site-updates of `iterations` red-black CG iterations in the paper's counting (Results,
    conventional Krylov solvers): an iteration applies M_pc and M_pc^dag, four half-lattice hops,
    which count as two full matrix multiplies of V5 = V4 * Ls site-updates each."""
    return FULL_MATMULS_PER_RB_ITERATION * V5 * iterations


FULL_MATMULS_PER_RB_ITERATION = 2

FORCE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_traffic.json")
FORCE_SOURCE = os.path.join(ROOT, "paper_2103_05034_amd", "csrc", "force.hip")
# the Ls = 16 force launches of the force workload (its Ls = 12 lattice takes the LDS-sum variant)
FORCE_KERNEL_PREFIX = "void dwf::force_dir_kernel<true>"


def measured_force_traffic(order):
    """HBM bytes per launch of the force kernel on the 16^3 x 32, Ls = 16 lattice from the
    rocprofv3 runs recorded in profiles/force_traffic.json for the traversal order `order`
    ({"mode": m[, "box": [..]]}), or None when force.hip changed since or no record has that order."""
    import hashlib

    try:
        rec = json.load(open(FORCE_TRAFFIC_FILE))
        digest = hashlib.sha256(open(FORCE_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("force_source_sha256") != digest:
        return None
    entry = rec.get("orders", {}).get(_order_key(order))
    return entry["bytes_per_launch"] if entry else None


def measured_traffic(key, order=None):
    """HBM bytes per hop launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs recorded in
    profiles/hop_traffic.json, or None when the hop kernel source changed since they were taken,
    or when they were taken in another traversal order than `order` ({"mode": m[, "box": [..]]})."""
    import hashlib

    try:
        rec = json.load(open(TRAFFIC_FILE))
        digest = hashlib.sha256(open(HOP_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("hop_source_sha256") != digest or key not in rec.get("workloads", {}):
        return None
    entry = rec["workloads"][key].get("orders", {}).get(_order_key(order) if order is not None else "", None)
    return entry["bytes_per_launch"] if entry else None


def _order_key(order):
    """'3:1,4,2' for boxes, '1' for mode 1: the key of a traffic record's traversal order."""
    return f"3:{','.join(map(str, order['box']))}" if order.get("mode") == 3 else str(order.get("mode", 0))


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def cpu_baseline_rb(cfg):
    """The oracle as it stands, one M_pc application on the workload's lattice."""
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import lattice as L

    dims, Ls = cfg["dims"], cfg["Ls"]
    U = synth.gauge_links(dims, cfg["eps"], seed=0)
    psi = L.on_parity(synth.gaussian_fermion(dims, Ls, seed=1), L.EVEN)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        L.mpc(U, psi, cfg["M5"], cfg["mf"])
        dt = time.perf_counter() - t0
    X, Y, Z, T = dims
    V5 = X * Y * Z * T * Ls
    return {
        "value": V5 / dt,
        "unit": "5D site-updates/s",
        "cores": 1,
        "host_cores": len(os.sched_getaffinity(0)),
        "kind": "oracle",
        "sample": f"one M_pc application (= {V5} site-updates by the paper's counting) of the FP64 NumPy oracle "
        f"on the {X}x{Y}x{Z}x{T}, Ls={Ls} lattice, BLAS limited to 1 thread; {dt:.1f} s",
    }


def run_rb_solve(args):
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    cfg = WORKLOADS["rb_solve"]
    dims, Ls = cfg["dims"], cfg["Ls"]
    X, Y, Z, T = dims
    V5 = X * Y * Z * T * Ls
    V5h = V5 // 2
    log("building inputs")
    U = torch.from_numpy(synth.gauge_links(dims, cfg["eps"], seed=0)).to("cuda")
    eta_nat = torch.from_numpy(synth.gaussian_fermion(dims, Ls, seed=1)[None]).to("cuda")
    op = dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=dwf.DWF_F64, max_nrhs=1, max_cg_rhs=1)
    if args.box:
        op.set_order_box(*(int(v) for v in args.box.split(",")))
        args.order = 3
    elif args.order >= 0:
        op.set_order(args.order)
    if args.tile:
        op.set_tile(args.tile, args.depth)
        tile = (args.tile, args.depth)
        if args.order < 0:  # pick the traversal order by timing M_pc^dag M_pc in the given tile
            args.order = _pick_order(op)
    elif args.order < 0:  # tile, depth and order together, timed on the solver itself
        spb, depth, args.order = _pick_shape_by_cg(op, dims, Ls)
        tile = (spb, depth)
    else:
        spb, depth, _ = op.autotune(1, 10)
        tile = (spb, depth)
    mode, box = op.get_order()
    order_desc = {"mode": mode, "box": list(box)} if mode == 3 else {"mode": mode}
    log(f"hop launch shape: {tile[0]} sites per workgroup, pipeline depth {tile[1]}, order {order_desc}")
    eta = op.pack(eta_nat, dwf.DWF_BOTH)
    del eta_nat
    psi = op.new_field(1, both=True)
    torch.cuda.synchronize()

    # pure operator throughput (outside the timed region): M_pc^dag M_pc applications
    v = op.new_field(1)
    w = op.new_field(1)
    op.pack(torch.from_numpy(synth.gaussian_fermion(dims, Ls, seed=2)[None]).to("cuda"), dwf.DWF_EVEN, out=v)
    for _ in range(3):
        op.mpcdagmpc(v, w)
    torch.cuda.synchronize()
    napp = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(napp):
        op.mpcdagmpc(v, w)
    e1.record()
    torch.cuda.synchronize()
    ms_app = e0.elapsed_time(e1) / napp
    log(f"M_pc^dag M_pc: {ms_app:.3f} ms per application")

    iters_all, res_all = [], []
    for k in range(args.warmup):
        psi.zero_()
        it, res = op.solve_rb(eta, psi, tol=1e-10, maxiter=20000)
        log(f"warmup {k}: {it} iterations, true residual {res:.2e}")
    torch.cuda.synchronize()
    # every HOP_SAMPLE-th hop launch carries an event pair: 5 is coprime with the four
    # passes of a CG iteration, so each pass kind is sampled equally often
    op.enable_timing(True, stride=HOP_SAMPLE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        psi.zero_()
        it, res = op.solve_rb(eta, psi, tol=1e-10, maxiter=20000)
        iters_all.append(it)
        res_all.append(res)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hop_ms, hop_launches = op.kernel_time()
    op.enable_timing(False)
    log(f"timed {args.steps} solves: {dt:.3f} s, iterations {iters_all}, residuals {res_all}")

    site_updates = sum(rb_site_updates(V5, it) for it in iters_all)
    value = site_updates / dt
    b1, b2 = hop_bytes_per_site(0, Ls)
    bytes_per_launch = cg_hop_bytes_per_launch(V5h, Ls)
    avg_ms = hop_ms / max(hop_launches, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "5D site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "red-black CG solve to 1e-10, FP64, 16^3x32 Ls=16 M5=1.8 mf=0.01, links exp(0.2iH)",
            "lattice": [X, Y, Z, T],
            "Ls": Ls,
            "M5": cfg["M5"],
            "mf": cfg["mf"],
            "tol": 1e-10,
            "cg_iterations": iters_all,
            "true_rel_residual": max(res_all),
            "parallelism": "single GPU",
            "hop_tile": {"sites_per_block": tile[0], "pipeline_depth": tile[1], "order": order_desc},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_traffic("rb_solve", order_desc),
            "kernel": "hop_kernel (all passes of the timed solves, every 5th launch timed; bytes = mean of a "
            "CG iteration's four)",
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": avg_ms,
            "launches": hop_launches,
            "timed_every": HOP_SAMPLE,
        },
        "context": {
            "paper_rb_cgnr_per_summit_node": 2.18e8,
            "note": "derived, not published: 6448 full matmuls in 62 s on 16^3x32x16 (4 V100, FP64, "
            "RBC configuration at m=0.001; Results, Krylov table); another machine and other links, so "
            "context only, not a baseline",
            "this_gpu_over_that_node": value / 2.18e8,
        },
        "operator": {
            "mpcdagmpc_ms": ms_app,
            "mpcdagmpc_site_updates_per_s": 2 * V5 / (ms_app * 1e-3),
            "mpcdagmpc_algorithmic_GBs": 2 * V5h * (b1 + b2) / (ms_app * 1e-3) / 1e9,
        },
    }
    op.close()
    return out


# traversal orders the bench tries: modes 0-2 and box cuts (nx, ny, nz) of the (x, y, z) volume
ORDER_CANDIDATES = [0, 1, 2, (1, 2, 4), (1, 4, 2), (1, 4, 4), (1, 2, 8), (1, 4, 8), (1, 3, 8), (1, 6, 4), (1, 6, 8),
                    (1, 8, 1), (1, 8, 8)]


def _set_order(op, cand):
    """Apply an ORDER_CANDIDATES entry; False when the lattice does not admit it."""
    import paper_2103_05034_amd as dwf

    try:
        if isinstance(cand, tuple):
            op.set_order_box(*cand)
        else:
            op.set_order(cand)
    except dwf.DWFError:
        return False
    return True


def _order_name(cand):
    return f"boxes {cand[0]}x{cand[1]}x{cand[2]}" if isinstance(cand, tuple) else str(cand)


def _pick_shape_by_cg(op, dims, Ls, iters=60):
    """Traversal order, then sites per workgroup and load-pipeline depth of the hop kernels,
    that make 60 FP64 CG iterations (the timed solve's own mix of passes) fastest, best of two
    timings each; orders a lattice does not admit are skipped."""
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    b = op.pack(torch.from_numpy(synth.gaussian_fermion(dims, Ls, seed=9)[None]).cuda(), dwf.DWF_EVEN)
    x = op.new_field(1)

    def time_cg():
        op.cg(b, x, 1, tol=1e-30, maxiter=10, allow_noconv=True)
        t = None
        for _ in range(2):
            x.zero_()
            tk, _ = _timed(lambda: op.cg(b, x, 1, tol=1e-30, maxiter=iters, allow_noconv=True))
            t = tk if t is None else min(t, tk)
        return t

    best = None
    op.set_tile(8, 3, 1)
    for cand in ORDER_CANDIDATES:
        if not _set_order(op, cand):
            continue
        t = time_cg()
        if best is None or t < best[0]:
            best = (t, cand)
    order = best[1]
    _set_order(op, order)
    best = None
    for spb in (4, 8, 16):
        for depth in (2, 3):
            op.set_tile(spb, depth, 1)
            t = time_cg()
            if best is None or t < best[0]:
                best = (t, spb, depth)
    _, spb, depth = best
    op.set_tile(spb, depth, 1)
    log(f"launch shape by CG timing: {spb} sites, depth {depth}, order {_order_name(order)} "
        f"({best[0] / iters * 1e3:.3f} ms per iteration)")
    return spb, depth, order


def _pick_order(op, reps=20):
    """Fastest site traversal order (ORDER_CANDIDATES) for M_pc^dag M_pc on the handle's lattice
    in its current launch shape; orders a lattice does not admit are skipped."""
    v = op.new_field(1)
    w = op.new_field(1)
    best = None
    for cand in ORDER_CANDIDATES:
        if not _set_order(op, cand):
            continue
        for _ in range(3):
            op.mpcdagmpc(v, w, 1)
        t, _ = _timed(lambda: [op.mpcdagmpc(v, w, 1) for _ in range(reps)])
        log(f"order {_order_name(cand)}: {t / reps * 1e3:.3f} ms per M_pc^dag M_pc")
        if best is None or t < best[0]:
            best = (t, cand)
    _set_order(op, best[1])
    return best[1]


def _timed(fn):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


def _fill_gaussian(op, buf, nvec, dims, Ls, seed, chunk=4):
    """Pack nvec complex Gaussian even fields into buf, a few at a time, drawn on the device
    (seeded per chunk, so handles of any precision receive the same fields)."""
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    fb = op.field_bytes(1)
    for k0 in range(0, nvec, chunk):
        n = min(chunk, nvec - k0)
        nat = synth.gaussian_fermion_device(dims, Ls, n, seed * 1000 + k0)
        op.pack(nat, dwf.DWF_EVEN, out=buf[k0 * fb : (k0 + n) * fb])
        torch.cuda.synchronize()
        del nat


def _setup_time(op, vecs, pristine, nvec, order, lo, hi, steps):
    """Chebyshev filter of nvec vectors + FP64-accumulated Gram-Schmidt, per step from the same input."""
    total = 0.0
    R = None
    for _ in range(steps):
        vecs.copy_(pristine)
        dt, R = _timed(lambda: (op.chebyshev_filter(vecs, nvec, order, lo, hi), op.gram_schmidt(vecs, nvec))[1])
        total += dt
    return total, R


def _roofline(bytes_per_launch, hop_ms, hop_n, kernel):
    avg = hop_ms / max(hop_n, 1)
    achieved = bytes_per_launch / (avg * 1e-3) / 1e9 if hop_n else 0.0
    return {
        "bound": "hbm",
        "achieved": achieved,
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": achieved / PEAK_HBM_GBS,
        "traffic": None,
        "kernel": kernel,
        "bytes_per_launch": bytes_per_launch,
        "avg_launch_ms": avg,
        "launches": hop_n,
    }


def cheb_step_bytes(prec, Ls, nrhs):
    """Algorithmic bytes per even 5D site and rhs of one Chebyshev step of M_pc^dag M_pc: four hop
    passes reading and writing 2 S, 3 S, 2 S and 5 S (the last also reads T_k and T_{k-1}),
    each with 8 L / (Ls nrhs) of links."""
    S, Lb = SPINOR_BYTES[prec], LINK_BYTES[prec]
    return 12 * S + 4 * 8.0 * Lb / (Ls * nrhs)


def mixed_cg_pass_bytes(Ls, prec_p):
    """Algorithmic bytes per even 5D site and rhs of the four hop passes of one low-precision CG
    iteration: p stored at prec_p (FP16 + scale or FP32), t, u and r in FP32, FP32 links.
    pass 1 reads p, writes t; pass 2 reads t and p, writes u; pass 3 reads u, writes t; pass 4
    reads t and u, reads and writes r; each reads 8 L / Ls of links."""
    Sp, S32, link = SPINOR_BYTES[prec_p], SPINOR_BYTES[1], 8.0 * LINK_BYTES[1] / Ls
    return (Sp + S32 + link, 2 * S32 + Sp + link, 2 * S32 + link, 4 * S32 + link)


def leg_batched(args, steps=3, warmup=1, fixed_order=False):
    """40 complex64 subspace vectors through the order-32 filter in one multi-rhs launch per pass,
    then FP64-accumulated Gram-Schmidt; compared with the same work in FP64 one vector at a time."""
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    cfg = WORKLOADS["batched"]
    dims, Ls, nvec = cfg["dims"], cfg["Ls"], cfg["nvec"]
    order, lo, hi = cfg["order"], cfg["lo"], cfg["hi"]
    X, Y, Z, T = dims
    V5h = X * Y * Z * T * Ls // 2
    U = torch.from_numpy(synth.gauge_links(dims, cfg["eps"], seed=0)).to("cuda")
    op = dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=dwf.DWF_F32, max_nrhs=nvec, max_cg_rhs=0)
    if fixed_order and args.box:  # a fixed traversal order (--workload batched, e.g. for counter runs)
        op.set_order_box(*(int(v) for v in args.box.split(",")))
    elif fixed_order and args.order >= 0:
        op.set_order(args.order)
    spb, depth, _ = op.autotune(nvec, 3)
    rpb = op.tile[2]
    mode, box = op.get_order()
    order_desc = {"mode": mode, "box": list(box)} if mode == 3 else {"mode": mode}
    log(f"batched FP32 autotune: spb={spb} depth={depth} rhs/workgroup={rpb} order {order_desc}")
    vecs = op.new_field(nvec)
    _fill_gaussian(op, vecs, nvec, dims, Ls, seed=2)
    pristine = vecs.clone()
    _setup_time(op, vecs, pristine, nvec, order, lo, hi, warmup)
    op.enable_timing(True)
    t_b, R_b = _setup_time(op, vecs, pristine, nvec, order, lo, hi, steps)
    hop_ms, hop_n = op.kernel_time()
    op.enable_timing(False)
    q_b = vecs[: op.field_bytes(2)].clone()
    # one filter step = 4 launches over nvec rhs
    per_launch = V5h * nvec * cheb_step_bytes(dwf.DWF_F32, Ls, nvec) / 4
    roof = _roofline(per_launch, hop_ms, hop_n, "hop_kernel, FP32, 40 rhs per launch (filter passes)")
    roof["traffic"] = measured_traffic("batched", order_desc)
    op.close()
    del op, vecs, pristine
    torch.cuda.empty_cache()
    log(f"batched: {steps} setups in {t_b:.3f} s")

    # FP64, one vector at a time
    op64 = dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=dwf.DWF_F64, max_nrhs=1, max_cg_rhs=0)
    op64.autotune(1, 3)
    v64 = op64.new_field(nvec)
    _fill_gaussian(op64, v64, nvec, dims, Ls, seed=2)
    p64 = v64.clone()
    _setup_time(op64, v64, p64, nvec, order, lo, hi, 1 if warmup else 0)
    n64 = max(1, steps // 2)
    t_64, R_64 = _setup_time(op64, v64, p64, nvec, order, lo, hi, n64)
    t_64 /= n64
    # agreement of the orthonormalised vectors (FP32 storage vs FP64)
    a = op64.unpack(v64[: op64.field_bytes(2)], 2, dwf.DWF_EVEN)
    op32 = dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=dwf.DWF_F32, max_nrhs=2, max_cg_rhs=0)
    b = op32.unpack(q_b, 2, dwf.DWF_EVEN)
    agree = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(a))
    op64.close()
    op32.close()
    del op64, op32, v64, p64, a, b
    torch.cuda.empty_cache()
    per_step = t_b / steps
    return {
        "value": nvec / per_step,
        "unit": "Chebyshev setup vecs/s",
        "higher_is_better": True,
        "ms_per_step": per_step * 1e3,
        "steps": steps,
        "dtype": "f32",
        "config": {
            "workload": "40 complex64 vectors, order-32 Chebyshev filter [0.05,60] of M_pc^dag M_pc in one "
            "multi-rhs launch per pass + FP64-accumulated Gram-Schmidt, 16^3x32 Ls=16",
            "autotuned_tile": {"sites_per_block": spb, "pipeline_depth": depth, "rhs_per_block": rpb,
                               "order": order_desc},
            "fp64_one_at_a_time_vecs_per_s": nvec / t_64,
            "speedup_vs_fp64_unbatched": t_64 / per_step,
            "fp32_vs_fp64_rel_diff_first_two_vectors": agree,
        },
        "roofline": roof,
    }


def run_batched(args):
    leg = leg_batched(args, max(args.steps, 1), args.warmup, fixed_order=True)
    return {"metric": METRIC, "n_gpus": 1, "warmup": args.warmup, "scaling": "weak", "vs_baseline": None,
            "data": "synthetic", **leg}


def leg_mixed(args):
    """Chebyshev setup of 24 vectors + 2 CG solves to 1e-10 at near-physical mass.

    Mixed: the setup runs on FP16 + per-site-scale fields (FP32 arithmetic, 24 vectors batched,
    FP64 Gram-Schmidt); the two solves run batched with the search direction in FP16 + scale,
    FP32 operator intermediates and residual, FP64 solution and reliable updates.  Plain: the
    same work in FP64, one vector / rhs at a time.  The same solves with an FP32 search
    direction are reported beside them."""
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    cfg = WORKLOADS["mixed"]
    dims, Ls, nvec = cfg["dims"], cfg["Ls"], cfg["nvec"]
    order, lo, hi = cfg["order"], cfg["lo"], cfg["hi"]
    X, Y, Z, T = dims
    V5h = X * Y * Z * T * Ls // 2
    log("mixed: building the 24^3x48 links")
    U = torch.from_numpy(synth.gauge_links(dims, cfg["eps"], seed=0)).to("cuda")

    def make(prec, nb, ncg):
        return dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=prec, max_nrhs=nb, max_cg_rhs=ncg)

    # two Gaussian sources, FP64 packed
    src = make(dwf.DWF_F64, 1, 0)
    fb = src.field_bytes(1, dwf.DWF_F64)
    b64 = torch.zeros(2 * fb, dtype=torch.uint8, device="cuda")
    _fill_gaussian(src, b64, 2, dims, Ls, seed=5, chunk=1)
    src.close()
    del src

    def setup(prec, nb):
        op = make(prec, nb, 0)
        spb, depth, _ = op.autotune(min(nb, 8), 2)
        vecs = op.new_field(nvec)
        _fill_gaussian(op, vecs, nvec, dims, Ls, seed=2)
        pristine = vecs.clone()
        log(f"setup prec={prec}: Chebyshev filter of {nvec} vectors (tile {spb}x{depth})")
        op.enable_timing(True)
        t, _ = _setup_time(op, vecs, pristine, nvec, order, lo, hi, 1)
        hop_ms, hop_n = op.kernel_time()
        op.enable_timing(False)
        log(f"setup prec={prec}: {t:.3f} s")
        per_launch = V5h * nb * cheb_step_bytes(prec, Ls, nb) / 4
        roof = _roofline(per_launch, hop_ms, hop_n, f"hop_kernel, {['FP64', 'FP32', 'FP16+scale'][prec]}, "
                         f"{nb} rhs per launch (filter passes)")
        op.close()
        del op, vecs, pristine
        torch.cuda.empty_cache()
        return t, [spb, depth], roof

    def solve(prec, batched, tag):
        op = make(prec, 2 if batched else 1, 2 if batched else 1)
        op.autotune(2 if batched else 1, 2)
        x64 = torch.zeros_like(b64)
        iters, res, codes = [], [], []
        op.set_progress(lambda it, rel: log(f"{tag} it={it} rel={max(rel):.2e}") and False, every=500)

        def run():
            chunks = [(0, 2)] if batched else [(0, 1), (1, 2)]
            for k0, k1 in chunks:
                code, it, r = op.cg(b64[k0 * fb : k1 * fb], x64[k0 * fb : k1 * fb], k1 - k0, tol=1e-10,
                                    maxiter=20000, allow_noconv=True)
                codes.append(code)
                iters.extend(it)
                res.extend(r)

        op.enable_timing(True)
        t, _ = _timed(run)
        hop_ms, hop_n = op.kernel_time()
        op.enable_timing(False)
        log(f"{tag}: {t:.3f} s, iterations {iters}, residuals {res}, status {codes}")
        op.close()
        del op, x64
        torch.cuda.empty_cache()
        return {"solve_s": t, "cg_iterations": iters, "true_rel_residual": res, "converged": not any(codes),
                "hop_ms": hop_ms, "hop_launches": hop_n}

    t_set_mixed, tile_mixed, roof_setup = setup(dwf.DWF_F16S, nvec)
    f16 = solve(dwf.DWF_F16S, True, "FP16-field CG")
    f32 = solve(dwf.DWF_F32, True, "FP32-field CG")
    t_set_plain, tile_plain, _ = setup(dwf.DWF_F64, 1)
    f64 = solve(dwf.DWF_F64, False, "FP64 CG")
    if not (f16["converged"] and f32["converged"] and f64["converged"]):
        raise SystemExit(f"a solve did not converge: FP16 {f16}, FP32 {f32}, FP64 {f64}")
    # the FP16-field solve's hop launches: the mean of the four passes over 2 rhs
    per_launch = 2 * V5h * sum(mixed_cg_pass_bytes(Ls, dwf.DWF_F16S)) / 4
    roof = _roofline(per_launch, f16.pop("hop_ms"), f16.pop("hop_launches"),
                     "hop_kernel of the FP16-field CG (2 rhs; p FP16+scale, t/u/r FP32; mean of the four passes)")
    for d in (f32, f64):
        d.pop("hop_ms"), d.pop("hop_launches")
    total_mixed = t_set_mixed + f16["solve_s"]
    total_plain = t_set_plain + f64["solve_s"]
    return {
        "value": total_plain / total_mixed,
        "unit": "x (plain FP64 time / mixed time), setup of 24 vectors + 2 CG solves to 1e-10",
        "higher_is_better": True,
        "ms_per_step": total_mixed * 1e3,
        "steps": 1,
        "dtype": "f16+scale storage, f32 arithmetic, f64 reliable updates and solution",
        "config": {
            "workload": "24^3x48 Ls=24 M5=1.8 mf=0.00078 links exp(0.15iH): Chebyshev setup of 24 vectors "
            "(order 32 [0.05,60]) + FP64 Gram-Schmidt + 2 CG solves to 1e-10",
            "mixed": {"setup_s": t_set_mixed, "setup_tile": tile_mixed, "setup_roofline": roof_setup, **f16},
            "plain_f64": {"setup_s": t_set_plain, "setup_tile": tile_plain, **f64},
            "fp32_field_solves": {**f32, "x_plain_over_mixed": total_plain / (t_set_mixed + f32["solve_s"])},
        },
        "roofline": roof,
    }


def run_mixed(args):
    leg = leg_mixed(args)
    return {"metric": METRIC, "n_gpus": 1, "warmup": 0, "scaling": "weak", "vs_baseline": None,
            "data": "synthetic", **leg}


def force_bytes(V4, Ls):
    """Algorithmic bytes of one force-kernel launch (both parities): a and b read once on each
    parity (4 FP64 half fields) and the gradient written, 4 links x 9 complex128 per 4D site."""
    return 4 * (V4 // 2) * Ls * SPINOR_BYTES[0] + V4 * 4 * 9 * 16


def run_force(args):
    """dS/dU of S = phi^dag (M_pc^dag M_pc)^-1 phi on 8^3 x 16, Ls = 12, FP64: CG, M_pc, force kernel;
    and the force kernel alone on the 16^3 x 32, Ls = 16 lattice, where its launch fills the chip,
    timed with HIP events against its algorithmic bytes."""
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    cfg = WORKLOADS["force"]
    dims, Ls = cfg["dims"], cfg["Ls"]
    U = torch.from_numpy(synth.gauge_links(dims, cfg["eps"], seed=0)).to("cuda")
    op = dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=dwf.DWF_F64, max_nrhs=1, max_cg_rhs=1)
    op.autotune(1, 5)
    phi = op.new_field(1)
    _fill_gaussian(op, phi, 1, dims, Ls, seed=3)
    X, Y = op.new_field(1), op.new_field(1)

    def step():
        X.zero_()
        _, it, res = op.cg(phi, X, 1, tol=1e-12, maxiter=100000, allow_noconv=True)
        op.mpc(X, Y, 1, False)
        return op.force(X, Y), it, res

    for _ in range(args.warmup):
        step()
    t, (G, it, res) = _timed(lambda: [step() for _ in range(args.steps)][-1])
    op.close()
    del op, U, phi, X, Y, G
    torch.cuda.empty_cache()

    # the force kernel on the 16^3 x 32, Ls = 16 lattice: dwf_force = two hop passes (Z, W) + the
    # force kernel; the hop passes are timed by the library's HIP events and subtracted
    c2 = WORKLOADS["rb_solve"]
    d2, L2 = c2["dims"], c2["Ls"]
    V4 = int(np.prod(d2))
    U2 = torch.from_numpy(synth.gauge_links(d2, c2["eps"], seed=0)).to("cuda")
    op2 = dwf.Operator(U2, d2, L2, c2["M5"], c2["mf"], prec=dwf.DWF_F64, max_nrhs=1, max_cg_rhs=1)
    op2.autotune(1, 3)
    X2, Y2 = op2.new_field(1), op2.new_field(1)
    _fill_gaussian(op2, X2, 1, d2, L2, seed=31)
    _fill_gaussian(op2, Y2, 1, d2, L2, seed=32)
    G2 = op2.force(X2, Y2)
    reps = 20
    by_order = {}
    best = None
    # the force kernel walks the sites in the handle's traversal order: time each order
    fixed = tuple(int(v) for v in args.box.split(",")) if args.box else (args.order if args.order >= 0 else None)
    for mode in ORDER_CANDIDATES if fixed is None else (fixed,):
        if not _set_order(op2, mode):
            continue
        op2.force(X2, Y2, G2)
        torch.cuda.synchronize()
        op2.enable_timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            op2.force(X2, Y2, G2)
        e1.record()
        torch.cuda.synchronize()
        hop_ms, hop_n = op2.kernel_time()
        op2.enable_timing(False)
        total_ms = e0.elapsed_time(e1)
        k_ms = (total_ms - hop_ms) / reps
        by_order[_order_name(mode)] = k_ms
        log(f"force kernel, order {_order_name(mode)}: {k_ms:.4f} ms ({total_ms / reps:.4f} ms per dwf_force)")
        if best is None or k_ms < best[0]:
            best = (k_ms, mode, total_ms, hop_ms)
    kernel_ms, order, total_ms, hop_ms = best
    nbytes = force_bytes(V4, L2)
    achieved = nbytes / (kernel_ms * 1e-3) / 1e9
    op2.close()
    return {
        "metric": METRIC,
        "value": args.steps / t,
        "unit": "force evaluations/s (CG to 1e-12 + M_pc + force kernel)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "pseudofermion force dS/dU, 8^3x16 Ls=12 mf=0.01, FP64",
            "cg_iterations": it,
            "true_rel_residual": res,
            "force_kernel_16x16x16x32_Ls16": {
                "dwf_force_ms": total_ms / reps,
                "hop_passes_ms": hop_ms / reps,
                "force_kernel_ms": kernel_ms,
                "order": _order_name(order),
                "force_kernel_ms_by_order": by_order,
            },
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_force_traffic({"mode": 3, "box": list(order)} if isinstance(order, tuple)
                                              else {"mode": order}),
            "kernel": "force_kernel, 16^3x32 Ls=16 (both parities; bytes: a, b on both parities + the gradient)",
            "bytes_per_launch": nbytes,
            "avg_launch_ms": kernel_ms,
            "launches": reps,
        },
    }


def run_operator(args):
    """M_pc^dag M_pc applications (args.steps of them, after args.warmup) on one lattice at one
    storage precision and rhs count, in the autotuned launch shape: the kernel-level view of the
    hop kernels for profiles, with a roofline from HIP events and the per-site bytes of a
    M_pc^dag M_pc (10 S + 32 L / (Ls nrhs) per even 5D site and rhs)."""
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    cfg = WORKLOADS["operator"]
    dims, Ls, eps = cfg["lattices"][args.lattice]
    prec = {"f64": dwf.DWF_F64, "f32": dwf.DWF_F32, "f16s": dwf.DWF_F16S}[args.prec]
    nrhs = args.nrhs
    X, Y, Z, T = dims
    V5h = X * Y * Z * T * Ls // 2
    U = torch.from_numpy(synth.gauge_links(dims, eps, seed=0)).to("cuda")
    op = dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=prec, max_nrhs=nrhs, max_cg_rhs=0)
    if args.box:
        op.set_order_box(*(int(v) for v in args.box.split(",")))
    elif args.order >= 0:
        op.set_order(args.order)
    spb, depth, _ = op.autotune(nrhs, 3)
    mode, box = op.get_order()
    log(f"operator: order {mode}{' boxes ' + 'x'.join(map(str, box)) if mode == 3 else ''}, tile {spb} x {depth}")
    v = op.new_field(nrhs)
    _fill_gaussian(op, v, nrhs, dims, Ls, seed=2)
    w = op.new_field(nrhs)
    for _ in range(args.warmup):
        op.mpcdagmpc(v, w, nrhs)
    torch.cuda.synchronize()
    op.enable_timing(True)
    t, _ = _timed(lambda: [op.mpcdagmpc(v, w, nrhs) for _ in range(args.steps)])
    hop_ms, hop_n = op.kernel_time()
    op.enable_timing(False)
    S, Lb = SPINOR_BYTES[prec], LINK_BYTES[prec]
    per_app = V5h * nrhs * (10 * S + 32.0 * Lb / (Ls * nrhs))
    op.close()
    return {
        "metric": METRIC,
        "value": 2 * V5h * 2 * nrhs * args.steps / t,
        "unit": "5D site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"M_pc^dag M_pc, {args.lattice} Ls={Ls}, {args.prec}, {nrhs} rhs per launch",
                   "tile": {"sites_per_block": spb, "pipeline_depth": depth},
                   "order": {"mode": mode, "box": list(box)} if mode == 3 else {"mode": mode}},
        "roofline": _roofline(per_app / 4, hop_ms, hop_n, f"hop_kernel, {args.prec}, {nrhs} rhs (mean of the 4 passes)"),
    }


def run_copy(args):
    """Device-to-device copy of a 4 GiB buffer: the known-size kernel that calibrates the
    FETCH_SIZE / WRITE_SIZE counters, and the practical copy ceiling of the box."""
    import torch

    n = WORKLOADS["copy"]["bytes"]
    x = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        y.copy_(x)
    t, _ = _timed(lambda: [y.copy_(x) for _ in range(args.steps)])
    gbs = 2 * n * args.steps / t / 1e9
    return {
        "metric": "device copy GB/s (read + write)",
        "value": gbs,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "copy of a 4 GiB buffer (counter calibration)"},
    }


def run_coarse(args):
    """Coarse-space transfer on 40 / 32 FP32 vectors at 16^3x32, Ls=16 with the Algorithm A / B
    blocks: chirality split, block orthonormalisation (two Cholesky-QR rounds), restriction and
    prolongation of one field, each timed and set against its algorithmic bytes."""
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    cfg = WORKLOADS["coarse"]
    dims, Ls = cfg["dims"], cfg["Ls"]
    X, Y, Z, T = dims
    V5h = X * Y * Z * T * Ls // 2
    S = SPINOR_BYTES[dwf.DWF_F32]
    U = torch.from_numpy(synth.gauge_links(dims, cfg["eps"], seed=0)).to("cuda")
    reps = max(args.steps, 1)
    results = {}
    for name, (block, nraw) in cfg["algos"].items():
        nvec = 2 * nraw
        op = dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=dwf.DWF_F32, max_nrhs=1, max_cg_rhs=0)
        nb = op.set_blocks(block)
        raw = op.new_field(nraw)
        _fill_gaussian(op, raw, nraw, dims, Ls, seed=2)
        basis = op.new_field(nvec)
        v = op.new_field(1)
        _fill_gaussian(op, v, 1, dims, Ls, seed=5, chunk=1)
        coarse = torch.zeros((1, nb, nvec), dtype=torch.complex128, device="cuda")
        out = op.new_field(1)
        steps = {
            "chiral_split": (lambda: op.chiral_split(raw, nraw, out=basis), 3 * nraw * S * V5h),
            "block_orthonormalize": (lambda: op.block_orthonormalize(basis, nvec), 6 * nvec * S * V5h),
            "restrict": (lambda: op.restrict(basis, nvec, v, 1, coarse=coarse), (nvec + 1) * S * V5h),
            "prolong": (lambda: op.prolong(basis, nvec, coarse, 1, out=out), (nvec + 1) * S * V5h),
        }
        res = {"block": list(block), "blocks": nb, "basis_vectors": nvec}
        for step, (fn, nbytes) in steps.items():
            for _ in range(args.warmup):
                fn()
            t, _ = _timed(lambda: [fn() for _ in range(reps)])
            ms = t / reps * 1e3
            res[step] = {"ms": ms, "algorithmic_GBs": nbytes / (ms * 1e-3) / 1e9}
            log(f"coarse {name} {step}: {ms:.3f} ms, {res[step]['algorithmic_GBs']:.0f} GB/s")
        # the transfer must stay a projector: restrict(prolong(c)) == c after orthonormalisation
        back = op.restrict(basis, nvec, out, 1)
        torch.cuda.synchronize()
        res["restrict_prolong_rel_err"] = float((back - coarse).abs().max() / coarse.abs().max())
        results[name] = res
        op.close()
        del op, raw, basis, v, out, coarse
        torch.cuda.empty_cache()
    a = results["A"]["restrict"]["algorithmic_GBs"]
    return {
        "metric": METRIC,
        "value": a,
        "unit": "GB/s (restriction of one field onto 40 FP32 basis vectors, 4x2x4x2 blocks)",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "ms_per_step": results["A"]["restrict"]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage, f64 sums",
        "data": "synthetic",
        "config": {"workload": "coarse-space transfer, 16^3x32 Ls=16, Algorithm A / B blocks", **results},
        "roofline": {
            "bound": "hbm",
            "achieved": a,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": a / PEAK_HBM_GBS,
            "traffic": None,
            "kernel": "block_dot_kernel (restriction)",
        },
    }


def run_krylov(args):
    """The Krylov table's FP64 rows on the 16^3x32, Ls=16 synthetic links: red-black CGNR with
    the first and the second Schur form, and unpreconditioned CGNR on D_DW^dag D_DW, all
    solving one D_DW psi = eta to 1e-10; iterations, full-lattice matrix multiplies (one
    red-black iteration or one CGNR iteration = 2) and time to solution."""
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    cfg = WORKLOADS["krylov"]
    dims, Ls = cfg["dims"], cfg["Ls"]
    X, Y, Z, T = dims
    V5 = X * Y * Z * T * Ls
    U = torch.from_numpy(synth.gauge_links(dims, cfg["eps"], seed=0)).to("cuda")
    op = dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=dwf.DWF_F64, max_nrhs=1, max_cg_rhs=2)
    op.autotune(1, 3)
    eta = op.pack(torch.from_numpy(synth.gaussian_fermion(dims, Ls, seed=1)[None]).cuda(), dwf.DWF_BOTH)
    rows = {}
    op.set_progress(lambda it, rel: log(f"  it={it} rel={rel[0]:.2e}") and False, every=1000)
    for name, form in (("prec-CGNR form 1", 1), ("prec-CGNR form 2", 2), ("CGNR unpreconditioned", 0)):
        psi = op.new_field(1, both=True)
        if form:
            op.set_schur_form(form)
            t, (it, res) = _timed(lambda: op.solve_rb(eta, psi, tol=cfg["tol"], maxiter=100000))
        else:
            op.set_schur_form(1)
            t, (it, res) = _timed(lambda: op.solve_unprec(eta, psi, tol=cfg["tol"], maxiter=100000))
        rows[name] = {"iterations": it, "full_matmuls": 2 * it, "time_s": t, "true_rel_residual": res,
                      "site_updates_per_s": 2 * V5 * it / t}
        log(f"{name}: {it} iterations, {t:.3f} s, residual {res:.2e}")
    op.close()
    base = rows["prec-CGNR form 1"]
    return {
        "metric": METRIC,
        "value": base["site_updates_per_s"],
        "unit": "5D site-updates/s (prec-CGNR form 1)",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": base["time_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Krylov table rows, 16^3x32 Ls=16 mf=0.01, links exp(0.2iH), tol 1e-10", **rows},
    }


def run_hdcr(args):
    """Two-level HDCR (Algorithm B: 2^4 x Ls blocks over both parities, 16 + 16 chiral basis
    vectors) on the 16^3x32, Ls=16 synthetic links at the light mass of the paper's HDCR tables
    (mf = 0.001): 16 Gaussian fields each low-pass filtered with T_300 of D^dag D over
    [0.05, 70] (the top of the interval above this lattice's lambda_max; the paper's recursive
    series from one Gaussian gives block-wise dependent vectors on these smooth links, whose
    light space has about a dozen modes), chirality split, block orthonormalisation and the
    little Dirac operator; then
    pGCR(H_DW) with the V(1,1) preconditioner (Chebyshev smoother [0.5, 70] of order 16, CGNR
    coarse solve to 0.02) to 1e-10, against the red-black CG solve of the same system.  The
    coarse matvec, which dominates the solve, is timed separately against its bytes."""
    import torch

    import paper_2103_05034_amd as dwf
    import synth

    cfg = WORKLOADS["hdcr"]
    dims, Ls = cfg["dims"], cfg["Ls"]
    X, Y, Z, T = dims
    V5 = X * Y * Z * T * Ls
    U = torch.from_numpy(synth.gauge_links(dims, cfg["eps"], seed=0)).to("cuda")
    op = dwf.Operator(U, dims, Ls, cfg["M5"], cfg["mf"], prec=dwf.DWF_F64, max_nrhs=1, max_cg_rhs=2)
    op.autotune(1, 3)
    eta = op.pack(torch.from_numpy(synth.gaussian_fermion(dims, Ls, seed=1)[None]).cuda(), dwf.DWF_BOTH)
    psi = op.new_field(1, both=True)
    t_rb, (it_rb, res_rb) = _timed(lambda: op.solve_rb(eta, psi, tol=cfg["tol"], maxiter=100000))
    log(f"red-black CG: {it_rb} iterations, {t_rb:.3f} s")
    nb = op.set_blocks(cfg["block"], both=True)
    nraw = cfg["nraw"]
    n = 2 * nraw
    hd = dwf.HDCR(op, n, smoother_order=cfg["smoother"][2], smoother_lo=cfg["smoother"][0],
                  smoother_hi=cfg["smoother"][1], coarse_tol=cfg["coarse_tol"], coarse_maxiter=5000,
                  nkrylov=cfg["nkrylov"])
    raw = op.new_field(nraw, both=True)
    fb = op.field_bytes(1)
    for k in range(nraw):  # field k of the both layout: even half k, odd half nraw + k
        one = op.pack(torch.from_numpy(synth.gaussian_fermion(dims, Ls, seed=300 + k)[None]).cuda(), dwf.DWF_BOTH)
        raw[k * fb : (k + 1) * fb] = one[:fb]
        raw[(nraw + k) * fb : (nraw + k + 1) * fb] = one[fb:]
    m, lo, hi = cfg["filter"]
    t_series, _ = _timed(lambda: hd.filter(raw, nraw, m, lo, hi))
    basis = op.new_field(n, both=True)
    t_ortho, _ = _timed(lambda: (op.chiral_split(raw, nraw, out=basis), op.block_orthonormalize(basis, n)))
    t_coarsen, _ = _timed(lambda: hd.set_basis(basis))
    log(f"setup: filter {t_series:.2f} s, split + orthonormalise {t_ortho:.2f} s, coarse operator {t_coarsen:.2f} s")
    steps = max(args.steps, 1)
    runs = []
    for _ in range(steps):
        psi = op.new_field(1, both=True)
        t, (it, res, ci) = _timed(lambda: hd.solve(eta, psi, tol=cfg["tol"], maxiter=500))
        runs.append((t, it, res, ci))
        log(f"HDCR: {it} outer, {ci} coarse iterations, {t:.3f} s, residual {res:.2e}")
    t, it, res, ci = min(runs)
    # the same solver with the little Dirac operator stored in complex64 (half the bytes per matvec)
    hd32 = dwf.HDCR(op, n, smoother_order=cfg["smoother"][2], smoother_lo=cfg["smoother"][0],
                    smoother_hi=cfg["smoother"][1], coarse_tol=cfg["coarse_tol"], coarse_maxiter=5000,
                    nkrylov=cfg["nkrylov"], coarse_prec=dwf.DWF_F32)
    hd32.set_basis(basis)
    runs32 = []
    for _ in range(steps):
        psi = op.new_field(1, both=True)
        t32, (it32, res32, ci32) = _timed(lambda: hd32.solve(eta, psi, tol=cfg["tol"], maxiter=500))
        runs32.append((t32, it32, res32, ci32))
        log(f"HDCR, complex64 coarse operator: {it32} outer, {ci32} coarse iterations, {t32:.3f} s, residual {res32:.2e}")
    t32, it32, res32, ci32 = min(runs32)
    x32, y32 = hd32.coarse_vector(), hd32.coarse_vector()
    for _ in range(3):
        hd32.coarse_apply(x32, y32)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        hd32.coarse_apply(x32, y32)
    e1.record()
    torch.cuda.synchronize()
    mv32_ms = e0.elapsed_time(e1) / 50
    hd32.close()
    # fine matrix multiplies (one D_DW each) per outer direction: 2 smoothers of order N
    # (N D^dag D + one H_DW each), 2 residuals of the cycle, and w = H_DW z
    N = cfg["smoother"][2]
    fine = it * (2 * (2 * N + 1) + 3)
    # the coarse matvec: 9 n x n complex blocks per coarse block, the input and the output
    x = hd.coarse_vector()
    y = hd.coarse_vector()
    for _ in range(3):
        hd.coarse_apply(x, y)
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        hd.coarse_apply(x, y)
    e1.record()
    torch.cuda.synchronize()
    mv_ms = e0.elapsed_time(e1) / reps
    mv_bytes = nb * 9 * n * n * 16 + 2 * nb * n * 16
    ach = mv_bytes / (mv_ms * 1e-3) / 1e9
    hd.close()
    # Algorithm A: larger blocks, more vectors, a smaller coarse grid (2048 blocks x 40)
    ca = cfg["algorithm_a"]
    nb_a = op.set_blocks(ca["block"], both=True)
    nraw_a, n_a = ca["nraw"], 2 * ca["nraw"]
    raw_a = op.new_field(nraw_a, both=True)
    for k in range(nraw_a):
        one = op.pack(torch.from_numpy(synth.gaussian_fermion(dims, Ls, seed=300 + k)[None]).cuda(), dwf.DWF_BOTH)
        raw_a[k * fb : (k + 1) * fb] = one[:fb]
        raw_a[(nraw_a + k) * fb : (nraw_a + k + 1) * fb] = one[fb:]
    hda = dwf.HDCR(op, n_a, smoother_order=cfg["smoother"][2], smoother_lo=cfg["smoother"][0],
                   smoother_hi=cfg["smoother"][1], coarse_tol=cfg["coarse_tol"], coarse_maxiter=5000,
                   nkrylov=cfg["nkrylov"], coarse_prec=dwf.DWF_F32)
    t_fa, _ = _timed(lambda: hda.filter(raw_a, nraw_a, m, lo, hi))
    basis_a = op.new_field(n_a, both=True)
    t_oa, _ = _timed(lambda: (op.chiral_split(raw_a, nraw_a, out=basis_a), op.block_orthonormalize(basis_a, n_a)))
    t_ca, _ = _timed(lambda: hda.set_basis(basis_a))
    psi = op.new_field(1, both=True)
    t_a, (it_a, res_a, ci_a) = _timed(lambda: hda.solve(eta, psi, tol=cfg["tol"], maxiter=500))
    log(f"HDCR Algorithm A (complex64 coarse operator): {it_a} outer, {ci_a} coarse iterations, {t_a:.3f} s, "
        f"residual {res_a:.2e}; setup {t_fa + t_oa + t_ca:.2f} s")
    hda.close()
    op.close()
    return {
        "metric": METRIC,
        "value": 1.0 / t,
        "unit": "HDCR solves/s (setup excluded), D_DW psi = eta to 1e-10",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": t * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "two-level HDCR (Algorithm B blocks, 32 chiral basis vectors), 16^3x32 Ls=16 mf=0.001, "
            "links exp(0.2iH), tol 1e-10",
            "blocks": nb,
            "basis_vectors": n,
            "outer_iterations": it,
            "coarse_iterations": ci,
            "coarse_iterations_per_cycle": ci / max(it, 1),
            "fine_matmuls": fine,
            "true_rel_residual": res,
            "solve_s": t,
            "setup_s": {"filter": t_series, "split_orthonormalize": t_ortho, "coarse_operator": t_coarsen},
            "red_black_cg": {"iterations": it_rb, "full_matmuls": 2 * it_rb, "time_s": t_rb, "true_rel_residual": res_rb,
                             "site_updates_per_s": 2 * V5 * it_rb / t_rb},
            "coarse_matvec_ms": mv_ms,
            "complex64_coarse_operator": {"outer_iterations": it32, "coarse_iterations": ci32, "solve_s": t32,
                                          "true_rel_residual": res32, "coarse_matvec_ms": mv32_ms},
            "algorithm_a_complex64": {"block": list(ca["block"]), "blocks": nb_a, "basis_vectors": n_a,
                                      "outer_iterations": it_a, "coarse_iterations": ci_a, "solve_s": t_a,
                                      "true_rel_residual": res_a,
                                      "setup_s": {"filter": t_fa, "split_orthonormalize": t_oa,
                                                  "coarse_operator": t_ca}},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": ach,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS,
            "traffic": None,
            "kernel": "coarse_matvec_kernel (little Dirac operator, %d blocks x 9 x %d^2 complex128)" % (nb, n),
            "bytes_per_launch": mv_bytes,
            "avg_launch_ms": mv_ms,
        },
    }


RUNNERS = {"batched": run_batched, "mixed": run_mixed, "force": run_force, "copy": run_copy, "coarse": run_coarse,
           "operator": run_operator,
           "krylov": run_krylov, "hdcr": run_hdcr}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rb_solve", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="default workload only: skip the batched and mixed legs")
    ap.add_argument("--lattice", default="16x16x16x32", choices=sorted(WORKLOADS["operator"]["lattices"]),
                    help="--workload operator: lattice")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "f16s"], help="--workload operator: storage")
    ap.add_argument("--nrhs", type=int, default=1, help="--workload operator: rhs per launch")
    ap.add_argument("--tile", type=int, default=0, help="sites per workgroup of the hop kernels (0 = autotune)")
    ap.add_argument("--depth", type=int, default=0, help="neighbour-load pipeline depth with --tile (0 = keep)")
    ap.add_argument("--order", type=int, default=-1,
                    help="site traversal order (0 lexicographic, 1 XCD octants, 2 XCD t-slabs; -1 = fastest)")
    ap.add_argument("--box", type=str, default="",
                    help="traversal order in boxes: the cut NX,NY,NZ of the (x, y, z) volume (overrides --order); "
                    "with --traffic, the order the counters were taken in")
    ap.add_argument(
        "--traffic",
        nargs=4,
        metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
        help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this bench and of --workload copy "
        "into profiles/hop_traffic.json (no GPU needed)",
    )
    ap.add_argument("--traffic-workload", default="rb_solve", choices=sorted(TRAFFIC_KERNELS),
                    help="with --traffic: the workload the counter runs were taken on")
    ap.add_argument(
        "--traffic-force",
        nargs=4,
        metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
        help="the same for the force kernel of --workload force, into profiles/force_traffic.json",
    )
    args = ap.parse_args()
    if args.traffic_force:
        import hashlib

        rec = summarize_traffic(*args.traffic_force, copy_bytes=WORKLOADS["copy"]["bytes"],
                                prefixes=[FORCE_KERNEL_PREFIX])
        order = ({"mode": 3, "box": [int(v) for v in args.box.split(",")]} if args.box
                 else {"mode": max(args.order, 0)})
        digest = hashlib.sha256(open(FORCE_SOURCE, "rb").read()).hexdigest()
        try:
            out = json.load(open(FORCE_TRAFFIC_FILE))
        except (OSError, ValueError):
            out = {}
        if out.get("force_source_sha256") != digest or "orders" not in out:
            out = {"force_source_sha256": digest, "orders": {}}
        out["orders"][_order_key(order)] = {"order": order, **rec}
        with open(FORCE_TRAFFIC_FILE, "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out["orders"][_order_key(order)], indent=1))
        return
    if args.traffic:
        import hashlib

        wl = args.traffic_workload
        rec = summarize_traffic(*args.traffic, copy_bytes=WORKLOADS["copy"]["bytes"],
                                prefixes=TRAFFIC_KERNELS[wl], last=TRAFFIC_LAST[wl])
        order = ({"mode": 3, "box": [int(v) for v in args.box.split(",")]} if args.box
                 else {"mode": max(args.order, 0)})
        digest = hashlib.sha256(open(HOP_SOURCE, "rb").read()).hexdigest()
        # one record per workload and traversal order, kept while the hop source is unchanged
        try:
            out = json.load(open(TRAFFIC_FILE))
        except (OSError, ValueError):
            out = {}
        if out.get("hop_source_sha256") != digest:
            out = {"hop_source_sha256": digest, "workloads": {}}
        out.setdefault("workloads", {}).setdefault(wl, {}).setdefault("orders", {})
        out["workloads"][wl]["orders"][_order_key(order)] = {"order": order, **rec}
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out["workloads"][wl]["orders"][_order_key(order)], indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(
            json.dumps({"error": "one GPU only: the library drives a single device (no domain decomposition across GPUs)"}),
            flush=True,
        )
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device visible"}), flush=True)
        sys.exit(1)
    if args.workload != "rb_solve":
        out = RUNNERS[args.workload](args)
    else:
        out = run_rb_solve(args)
        if not args.no_cpu_baseline:
            log("timing the oracle (cpu baseline)")
            out["cpu_baseline"] = cpu_baseline_rb(WORKLOADS["rb_solve"])
        if not args.no_legs:
            # the metric's other parts, each on its own workload with its own roofline
            out["legs"] = {}
            log("leg: batched Chebyshev setup (16^3x32, Ls 16, 40 FP32 vectors)")
            out["legs"]["batched"] = leg_batched(args)
            log("leg: FP64 vs mixed setup + 2 solves (24^3x48, Ls 24, mf 0.00078)")
            out["legs"]["mixed"] = leg_mixed(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
