#!/usr/bin/env python3
"""Throughput of the per-step FAS solve of the second-order CHHS scheme on one GPU.

One "step" is one time step of (2.4)-(2.7) for every instance: setup, FAS
V(2,2) cycles to the residual tolerance, the post-step reductions (mass, E_h,
F_h, dissipation terms) and the state rotation, all through the C ABI of
libchhs (chhs_step_log: the reductions run every step).

The default workload is the ragged batch: 64 independent 2D instances, 16 each
of 128^2, 256^2, 512^2 and 1024^2 on (0,1)^2, eps ~ U[0.01, 0.05],
gamma ~ U[0.5, 5], s in {1e-4, 5e-4}, phi0 = m + 0.05 (2U - 1), m ~ U[-0.3, 0.3],
advanced together by the batched mixed-precision path (FP32 inner V-cycles,
FP64 residual, correction and reductions, graph-replayed cycles) and, beside it,
by the plain FP64 path as a sequential loop over single-instance contexts.
The single-grid 2D FP64 spinodal workload at 2048^2 is measured too and
reported under extra keys.  ``--workload`` selects another single workload.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import contextlib
import gc
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FAS cell-updates/s + HBM roofline %; batched FP32+refine vs plain FP64 at tol"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 256 << 20
BATCHED = "batched-64-2d-mixed"
# worker processes of the oracle's process pool (the machine's CPU share)
MAX_POOL = 16


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def launch_bytes_per_cell(dim, cls, mixed=False, kind=None):
    """Algorithmic bytes per finest cell of one finest-level launch of a kernel class.

    FP64 plain path (8 B per value).  On the finest level f_phi = phi^m and
    f_p = 0, so a smoothing step reads phi, mu, p, phi_*, phi^m, f_mu and writes
    phi, mu, p.
      2D pre0  : one launch = nu1 fused steps + residual + restriction:
                 6 reads + 3 writes, plus u_c, ub_c and R(r) written on the
                 coarse grid (9 values per 4 fine cells)                    = 90 B
      2D post0 : one launch = prolongation + nu2 fused steps + norm partials:
                 6 reads + 3 writes, plus u_c, ub_c read (6 per 4 cells)    = 84 B
      3D       : one launch = one color of one step: the other color's phi,
                 mu, p, phi_* (4 values per 2 cells), the color's phi, phi_*,
                 phi^m, f_mu (4 per 2 cells; f_phi = phi^m and f_p = 0 are not
                 read) and its new phi, mu, p (3 per 2 cells)               = 44 B
      3D fused (kind "zmarch"): one launch = one whole step: u, phi_*, phi^m
                 and f_mu read (f_phi = phi^m, f_p = 0 are not), u written:
                 (6 + 3) values                                             = 72 B
    Mixed precision, FP32 correction form (4 B per value; general right-hand
    sides and the base state b on every level):
      2D pre0  : 9 reads + 3 writes, plus u_c, ub_c, R(r), b_c (10 per 4)   = 58 B
      2D post0 : 9 reads + 3 writes, plus u_c, ub_c read (6 per 4)          = 54 B
      3D       : (4 + 7 + 3) values per 2 cells                             = 28 B
      3D fused : u, phi_*, phi^m, f, b read, u written: (9 + 3) values      = 48 B
      refine   : the FP64 refinement launch: u (FP64), e (FP32), phi_*,
                 phi^m, f_mu (FP64) read; u + e (FP64), the three FP32
                 right-hand sides and b written:
                 24 + 12 + 24 + 24 + 12 + 4                                 = 100 B
                 (the step's setup forms the first right-hand side itself)
    """
    if cls == "refine":
        return 100.0
    if mixed:
        if dim == 2:
            return {"pre0": (12 + 10 / 4) * 4, "post0": (12 + 6 / 4) * 4}[cls]
        return (9 + 3) * 4 if kind == "zmarch" else (4 + 7 + 3) / 2 * 4
    if dim == 2:
        return {"pre0": (9 + 9 / 4) * 8, "post0": (9 + 6 / 4) * 8}[cls]
    return (6 + 3) * 8 if kind == "zmarch" else (4 + 4 + 3) / 2 * 8


SWEEP_KEYS = ("nu1", "nu2", "nu1_coarse", "nu2_coarse", "prolong", "inner_cycles")


def vcycle_bytes(dim, shape, level_kernels, sweeps=None):
    """Algorithmic bytes of one FP64 V-cycle over every level.

    sweeps: (nu1, nu2, nu1_coarse, nu2_coarse, prolong[, inner_cycles]) as chhs_tune_sweeps
    reports them (default V(2,2), piecewise-constant prolongation).  Per cell
    of level l (n_l cells, r = 2^dim children per coarse cell, 8 B per value),
    what each launch of the cycle must move at minimum; a fused 2D launch
    takes up to two smoothing steps, so nu steps take ceil(nu / 2) launches:
      every fused launch          : u, phi_*, phi^m and the right-hand sides
                                    read (finest level: f_mu only, 6 values;
                                    coarse levels: f, 8 values), u written (3)
      first pre launch, coarse    : reads the restricted residual fr and writes
                                    f = fr + N(u) as well (+ 3)
      last pre launch             : writes u_c, ub_c and R(r) on level l + 1
                                    (+ 9/r)
      first post launch           : reads u_c and ub_c to prolong (+ 6/r); with
                                    the bilinear prolongation a launch of its
                                    own instead (u read and written, u_c, ub_c
                                    read: 6 + 6/r)
      strips on a coarse level    : a separate launch forms f (u, fr, phi_*,
                                    phi^m read, f written: 11), the first launch
                                    then reads f (no + 3)
      per-cell kernels            : 2 (nu1 + nu2) color launches of 52 B (44 B
                                    on the finest level); the
                                    residual + restriction (8 + 9/r); the
                                    right-hand side of level l + 1 unless the
                                    tail forms it, 11/r; the prolongation
                                    (6 + 6/r)
      fused 3D steps ("zmarch")   : nu1 + nu2 launches of 88 B (72 B on the
                                    finest level, which reads no f_phi, f_p),
                                    the transfers as for per-cell kernels
      (3D, either kind: on the finest level of an instance of at least 2^20
      cells the residual + restriction runs by z marching and reads 6 values,
      not 8)
      tail (one launch)           : u and fr of its top level read, u written,
                                    phi_* and phi^m of every tail level read
    The norm reduction and the per-cycle readback (a few KB) are left out.
    """
    nu1, nu2, nu1c, nu2c, prolong = tuple(sweeps)[:5] if sweeps is not None else (2, 2, 0, 0, 0)
    nu1c = nu1c or nu1
    nu2c = nu2c or nu2
    r = 2 ** dim
    n0 = 1
    for s in shape:
        n0 *= s
    kinds = [k[0] if isinstance(k, (list, tuple)) else k for k in level_kernels]
    total = 0.0
    for l, kind in enumerate(kinds):
        n = n0 / r ** l
        a, b = (nu1, nu2) if l == 0 else (nu1c, nu2c)
        if kind == "tail":
            rest = sum(n0 / r ** k for k in range(l, len(kinds)))
            total += 8 * (9 * n + 2 * rest)
            break
        if kind in ("per-cell", "zmarch"):
            next_tail = l + 1 < len(kinds) and kinds[l + 1] == "tail"
            smooth = ((a + b) * 2 * (44 if l == 0 else 52) / 8 if kind == "per-cell"
                      else (a + b) * (9 if l == 0 else 11))
            # the residual + restriction from the finest level of an instance
            # of at least 2^20 cells runs by z marching and reads no f_phi, f_p
            zres = dim == 3 and l == 0 and n0 >= 2 ** 20
            v = smooth + ((6 if zres else 8) + 9 / r) + (6 + 6 / r)
            v += 0 if next_tail else 11 / r
        else:
            read = 6 if l == 0 else 8
            pre = -(-a // 2) * (read + 3) + 9 / r
            if l > 0:
                pre += 11 if kind == "strips" else 3
            post = -(-b // 2) * (read + 3)
            post += (6 + 6 / r) if prolong == 1 else 6 / r
            v = pre + post
        total += 8 * v * n
    return total


# HBM traffic measured with rocprofv3 counters, one record per workload; a
# record lists the sources of the kernels it covers and is reported only while
# they hash as they did when the counters were taken.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash(sources):
    import hashlib
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, cls, level0_kernel):
    """The committed counter record of a launch class of a workload: the scaled
    FETCH_SIZE + WRITE_SIZE bytes per launch and the algorithmic bytes of the
    same launches, or None if there is no record for this workload and class,
    the finest level runs another kernel configuration, or the kernel sources
    changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            recs = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = recs.get(workload)
    if rec is None or rec.get("source_sha256") != kernel_source_hash(rec.get("sources", [])):
        return None
    # the finest level must run the same kind of kernel (tiles, strips, fused 3D
    # step); the autotuned block size or segment height may differ between runs
    if list(rec.get("level0_kernel", [None]))[:1] != list(level0_kernel)[:1]:
        return None
    return rec.get("launches", {}).get(cls)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_info():
    return {"cpu": cpu_model(), "os_cpu_count": os.cpu_count(),
            "omp_threads": os.environ.get("OMP_NUM_THREADS")}


# ---- the oracle on the host ------------------------------------------------------------

def _oracle_step(job):
    """One oracle time step of one instance (worker of the process pool), with
    the cycle (sweeps per level, prolongation) the GPU context of that instance
    uses."""
    import numpy as np
    from oracle import fas, scheme
    prev, cur, mu, p, eps, gamma, s, h, cyc = job
    prm = scheme.Params(eps=eps, gamma=gamma, s=s, h=h)
    nu1, nu2, nu1c, nu2c, prolong = tuple(cyc)[:5]
    opts = fas.Opts(tol=1e-10, nu1=nu1, nu2=nu2, nu1_coarse=nu1c, nu2_coarse=nu2c,
                    prolong="bilinear" if prolong == 1 else "constant")
    t0 = time.perf_counter()
    r = fas.solve_step(prev, cur, mu, p, prm, opts)
    return np.asarray(r.phi), r.vcycles, time.perf_counter() - t0


@contextlib.contextmanager
def no_gc():
    """Python's cyclic collector off while a region is timed (as timeit does):
    a full collection over the interpreter's objects takes tens of
    milliseconds and would otherwise land in whichever region it falls in."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


def make_pool(workers):
    """A pool of single-threaded worker processes, forked before this process
    touches the GPU (the workers run NumPy only)."""
    import multiprocessing as mp
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    return mp.get_context("fork").Pool(workers)


def oracle_sample(phi_prev, phi_cur, mu, p, w, cycles_per_step, max_cells=1 << 22):
    """Time the oracle on a bounded sample of one step: setup, three V-cycles
    and one residual evaluation; return (cell-updates/s estimate, description,
    wall seconds).  Grids above max_cells are sampled on their leading box of
    halved extents (same spacing h) so that the sample stays within tens of
    seconds of CPU work; the oracle's cost per cell does not depend on the
    grid's size."""
    import numpy as np
    from oracle import fas, scheme
    grid = phi_cur.shape
    n = grid[-1]
    k = 0
    while int(np.prod([e >> k for e in grid])) > max_cells:
        k += 1
    if k:
        box = tuple(slice(0, e >> k) for e in grid)
        phi_prev, phi_cur, mu, p = (np.ascontiguousarray(a[box]) for a in (phi_prev, phi_cur, mu, p))
    prm = scheme.Params(eps=w["eps"], gamma=w["gamma"], s=w["s"], h=1.0 / n)
    t0 = time.perf_counter()
    phi_star, f = scheme.step_rhs(phi_prev, phi_cur, prm)
    levels = fas.build_levels(phi_star, phi_cur.copy(), f, prm.h)
    u = [phi_cur.copy(), mu.copy(), p - np.mean(p)]
    us = [None] * len(levels)
    us[0] = u
    t1 = time.perf_counter()
    scheme.residual_norm(scheme.residual(u, f, levels[0], prm), prm.h)
    t2 = time.perf_counter()
    ncyc = 3
    for _ in range(ncyc):
        fas.vcycle(levels, us, 0, prm, fas.Opts())
    t3 = time.perf_counter()
    t_cycle = (t3 - t2) / ncyc
    t_step = (t1 - t0) + (t2 - t1) * (cycles_per_step + 1) + t_cycle * cycles_per_step
    where = ("x".join(str(e) for e in phi_cur.shape) + " leading box of " if k else "") + \
        "x".join(str(e) for e in grid)
    desc = (f"oracle on the first timed step's input at {where}: setup {t1 - t0:.2f}s, one "
            f"residual {t2 - t1:.2f}s, {ncyc} V(2,2) cycles {t3 - t2:.2f}s; step time = setup + "
            f"{cycles_per_step:.2f} x (cycle + residual) + residual, with the GPU's mean "
            f"V-cycles per step")
    return phi_cur.size / t_step, desc, t3 - t0


# ---- timing helpers ----------------------------------------------------------------------

def dominant_class(tim, classes):
    """The kernel class with the largest device time among those timed."""
    return max(classes, key=lambda k: tim[k][0])


def roofline_record(cls, tim, bytes_per_launch, name, traffic):
    """The roofline object of the timed class.  traffic: the class's counter
    record (or None); its ratio of counted to algorithmic bytes, measured on
    full-batch launches, scales this run's algorithmic bytes per launch."""
    ms_k, n_k = tim[cls]
    avg = ms_k / 1e3 / max(1, n_k)
    achieved = bytes_per_launch / avg / 1e9 if n_k else 0.0
    ratio = None if traffic is None else (traffic["bytes_per_launch"]
                                          / traffic["algorithmic_bytes_per_launch"])
    rec = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": None if traffic is None else round(ratio * bytes_per_launch),
           "kernel": name, "avg_launch_us": round(avg * 1e6, 2), "launches": n_k,
           "algorithmic_bytes_per_launch": round(bytes_per_launch)}
    if traffic is not None:
        rec["traffic_record"] = traffic
        rec["traffic_ratio"] = round(ratio, 3)
    return rec


# ---- the batched workload ----------------------------------------------------------------

def run_batched(args, pool):
    """64 ragged 2D instances by the batched mixed-precision path, against the
    plain FP64 path as a sequential loop over single-instance contexts (same
    library, same inputs, the reductions every step on both sides)."""
    import numpy as np
    import torch
    from paper_1611_02967_amd import chhs
    from workloads import batched_instances

    insts = batched_instances(count=64)
    probs = [chhs.make_problem(it.shape, it.h, it.eps, it.gamma, it.s) for it in insts]
    phi0s = [it.phi0() for it in insts]
    sizes = [int(np.prod(it.shape)) for it in insts]
    cells = sum(sizes)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    log(f"{BATCHED}: {len(insts)} instances, {cells} cells")

    flat = np.concatenate([a.ravel() for a in phi0s])
    tp = torch.from_numpy(flat).cuda()
    tc = tp.clone()
    tm = torch.zeros_like(tp)
    tpp = torch.zeros_like(tp)
    # the warm-up steps time the finest-level FP32 smoothing launches and the
    # FP64 refinement launch; the timed region times only the dominant one
    cand = ("pre0", "post0", "refine")
    sv = chhs.Solver(probs, chhs.chhs_default_opts(tol=1e-10, precision=1,
                                                   timing=chhs.timing_mask(*cand),
                                                   smoother=args.smoother,
                                                   autotune=int(args.autotune),
                                                   inner_cycles=args.inner_cycles))
    sweeps = None
    if args.tune_sweeps:
        # sweeps per level, prolongation and FP32 cycles per refinement by time
        # to tolerance on the first step's system (the state is not advanced),
        # before the warm-up steps, which then run the kept cycle
        sweeps = sv.tune_sweeps(tp, tc, tm, tpp)
        log(f"tuned {SWEEP_KEYS} = {sweeps}")
    inner = max(1, sweeps[5] if sweeps is not None else args.inner_cycles)
    sv.timing(reset=True)
    for k in range(args.warmup):
        _, lg = sv.step_log(tp, tc, tm, tpp, 1)
        log(f"warmup step {k + 1}/{args.warmup}: max {max(x['vcycles'] for x in lg[0])} "
            f"refinement steps")
    tim_w = sv.timing(reset=True)
    cls = dominant_class(tim_w, cand)
    sv.set_timing(chhs.timing_mask(cls))
    torch.cuda.synchronize()
    start = [t.clone() for t in (tp, tc, tm, tpp)]
    start_host = [t.cpu().numpy() for t in start]

    torch.cuda.synchronize()
    with no_gc():
        t0 = time.perf_counter()
        _, lg = sv.step_log(tp, tc, tm, tpp, args.steps)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    tim = sv.timing()
    refine = [[rec["vcycles"] for rec in step] for step in lg]
    total_refine = sum(sum(r) for r in refine)
    log(f"batched mixed: {args.steps} steps in {elapsed:.3f}s, {total_refine} instance "
        f"refinement steps")
    f_ok = all(lg[m][i]["F_h"] <= (lg[m - 1][i]["F_h"] if m else np.inf) + 1e-12
               for m in range(len(lg)) for i in range(len(insts)))

    # algorithmic bytes of the timed class's launches in the timed region: each
    # launch covers the instances still active in that refinement step
    if cls == "refine":
        per_launch_cells = sum(
            sizes[i] * refine[m][i] for m in range(args.steps) for i in range(len(insts))) * 100
        bytes_launch = per_launch_cells / max(1, tim[cls][1])
        name = ("finest-level FP64 refinement launch over the batch (u += e, residual of "
                "(2.5)-(2.7), FP32 right-hand side and base state, norm partials)")
    else:
        # every refinement of an instance runs `inner` FP32 cycles; the first
        # pre launch of each starts from a zero correction and reads no u
        active_cells = sum(sizes[i] * refine[m][i] for m in range(args.steps)
                           for i in range(len(insts)))
        per_ref = inner * launch_bytes_per_cell(2, cls, mixed=True)
        if cls == "pre0":
            per_ref -= 12.0
        bytes_launch = per_ref * active_cells / max(1, tim[cls][1])
        name = (f"finest-level FP32 {'pre' if cls == 'pre0' else 'post'}-smoothing launch "
                f"over the batch (correction form)")
    level_kernels = [list(k) for k in sv.level_kernels()]
    traffic = measured_traffic(BATCHED, cls, level_kernels[0])
    roofline = roofline_record(cls, tim, bytes_launch, name, traffic)
    others = {}
    for k in cand:
        if k != cls and tim_w[k][1]:
            others[k] = {"avg_launch_us_warmup": round(tim_w[k][0] / tim_w[k][1] * 1e3, 2),
                         "launches_warmup": tim_w[k][1]}
    roofline["other_classes"] = others

    # per-class device time per step from the same start state, every class
    # timed (outside the timed region)
    kernel_ms = {}
    if not args.no_breakdown:
        extra = (dict(inner_cycles=args.inner_cycles) if sweeps is None
                 else dict(zip(SWEEP_KEYS, sweeps)))
        sb = chhs.Solver(probs, chhs.chhs_default_opts(tol=1e-10, precision=1, timing=1,
                                                       smoother=args.smoother,
                                                       autotune=int(args.autotune), **extra))
        st_b = [t.clone() for t in start]
        sb.step_log(*st_b, 1)
        sb.timing(reset=True)
        nb = 2
        sb.step_log(*st_b, nb)
        kernel_ms = {k: round(v[0] / nb, 4) for k, v in sb.timing().items() if v[1]}
        sb.close()
        del st_b

    # the sequential plain FP64 loop: one context per instance, one step each
    # per round, with the reductions every step
    seq = [] if args.no_sequential else [
        chhs.Solver(pr, chhs.chhs_default_opts(tol=1e-10, precision=0, smoother=args.smoother,
                                               autotune=int(args.autotune)))
        for pr in probs]
    views = lambda ts, i: [t[offs[i]:offs[i + 1]] for t in ts]
    sp = [t.clone() for t in start]
    seq_sweeps = {}
    for i, s1 in enumerate(seq):       # warm-up: one step each (graph capture)
        if args.tune_sweeps:
            ch = s1.tune_sweeps(*views(sp, i))
            seq_sweeps[str(ch)] = seq_sweeps.get(str(ch), 0) + 1
        s1.step_log(*[v.clone() for v in views(sp, i)], 1)
    torch.cuda.synchronize()
    with no_gc():
        t0 = time.perf_counter()
        seq_cycles = 0
        for _ in range(args.steps):
            for i, s1 in enumerate(seq):
                _, lq = s1.step_log(*views(sp, i), 1)
                seq_cycles += lq[0][0]["vcycles"]
        torch.cuda.synchronize()
        elapsed_seq = max(time.perf_counter() - t0, 1e-12)
    log(f"sequential fp64: {args.steps} rounds in {elapsed_seq:.3f}s, {seq_cycles} V-cycles")

    # one step of both paths from the timed region's start state
    a = [t.clone() for t in start]
    sv.step(*a, 1)
    mixed_phi = a[1].cpu().numpy()
    err = 0.0
    fp64_phi = []
    for i, s1 in enumerate(seq):
        b = [v.clone() for v in views(start, i)]
        s1.step(*b, 1)
        fp64_phi.append(b[1].cpu().numpy())
        err = max(err, float(np.max(np.abs(mixed_phi[offs[i]:offs[i + 1]] - fp64_phi[i]))))
    log(f"max |phi_mixed - phi_fp64| over instances after one step: {err:.2e}")
    seq_cycles_opts = []
    for s1 in seq:
        o = s1.get_opts()
        seq_cycles_opts.append((o.nu1, o.nu2, o.nu1_coarse, o.nu2_coarse, o.prolong))
        s1.close()
    sv.close()

    inst_steps = len(insts) * args.steps
    out = {
        "metric": METRIC,
        "value": cells * args.steps / elapsed,
        "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": BATCHED, "instances": len(insts),
                   "grids": [128, 256, 512, 1024], "cells": cells, "eps": "U[0.01,0.05]",
                   "gamma": "U[0.5,5]", "s": "{1e-4,5e-4}", "tol": 1e-10, "cycle": "V(2,2)",
                   "precision": "fp32 inner + fp64 refinement",
                   "inner_cycles": inner,
                   "reductions": "mass, E_h, F_h, dissipation every step"},
        "instance_steps_per_s": inst_steps / elapsed,
        "refinement_steps_per_instance_step": total_refine / inst_steps,
        "sequential_fp64": {"value": cells * args.steps / elapsed_seq,
                            "unit": "cell-updates/s",
                            "instance_steps_per_s": inst_steps / elapsed_seq,
                            "ms_per_round": elapsed_seq / args.steps * 1e3,
                            "vcycles_per_instance_step": seq_cycles / inst_steps} if seq else None,
        "max_abs_err_phi_vs_fp64": err if seq else None,
        "speedup_vs_sequential_fp64": elapsed_seq / elapsed if seq else None,
        "energy_F_nonincreasing": bool(f_ok),
        "level_kernels": level_kernels,
        "sweeps": None if sweeps is None else dict(zip(SWEEP_KEYS, sweeps)),
        "sequential_fp64_sweeps": seq_sweeps or None,
        "kernel_ms_per_step": kernel_ms,
        "roofline": roofline,
    }

    if pool is not None and seq:
        # the oracle: one time step of instances 0..7 (two of each grid size)
        # from the timed region's start state, in the process pool
        sample = list(range(8))
        jobs = []
        for i in sample:
            it = insts[i]
            sl = slice(offs[i], offs[i + 1])
            jobs.append(tuple(x[sl].reshape(it.shape).copy() for x in start_host)
                        + (it.eps, it.gamma, it.s, it.h, seq_cycles_opts[i]))
        log(f"timing the oracle: one step of instances {sample[0]}..{sample[-1]} in a pool of "
            f"{pool._processes} processes")
        import resource
        ru0 = resource.getrusage(resource.RUSAGE_CHILDREN)
        t0 = time.perf_counter()
        res = pool.map(_oracle_step, jobs, chunksize=1)
        wall = time.perf_counter() - t0
        ru1 = resource.getrusage(resource.RUSAGE_CHILDREN)
        worker_s = sum(r[2] for r in res)
        sample_cells = sum(sizes[i] for i in sample)
        err_or = max(float(np.max(np.abs(mixed_phi[offs[i]:offs[i + 1]] - res[k][0].ravel())))
                     for k, i in enumerate(sample))
        err_or64 = max(float(np.max(np.abs(fp64_phi[i] - res[k][0].ravel())))
                       for k, i in enumerate(sample))
        out["cpu_baseline"] = {
            "value": sample_cells / wall, "unit": "cell-updates/s", "cores": pool._processes,
            "kind": "oracle",
            "sample": (f"one time step (FAS to tol 1e-10, each instance with the sweeps its FP64 "
                       f"GPU context uses) of instances {sample[0]}-"
                       f"{sample[-1]} of the batch ({sample_cells} cells: two each of 128^2, "
                       f"256^2, 512^2, 1024^2) from the timed region's start state, single-threaded "
                       f"NumPy per process, {pool._processes} processes; value = cells / wall"),
            "wall_s": round(wall, 2), "worker_cpu_s": round(worker_s, 2),
            "children_cpu_s": round((ru1.ru_utime + ru1.ru_stime) - (ru0.ru_utime + ru0.ru_stime), 2),
            "host": host_info()}
        out["parity"] = {"instances": sample, "steps": 1,
                         "max_abs_err_phi_mixed_vs_oracle": err_or,
                         "max_abs_err_phi_fp64_vs_oracle": err_or64}
        log(f"oracle: {sample_cells / wall:.3e} cell-updates/s ({wall:.1f}s wall); "
            f"max|phi_mixed - oracle| = {err_or:.2e}, max|phi_fp64 - oracle| = {err_or64:.2e}")
    return out


# ---- one grid ---------------------------------------------------------------------------

def run_single(args, name, cpu_baseline=True, parity=True, breakdown=True, copy_calibration=False):
    """One named workload (one grid) through chhs_step_log; returns the record."""
    import numpy as np
    import torch
    from paper_1611_02967_amd import chhs
    from workloads import WORKLOADS, uniform_field

    w = WORKLOADS[name]
    n, dim = w["n"], w["dim"]
    shape = (n,) * dim
    cells = n ** dim
    log(f"workload {name}: {shape}, eps {w['eps']}, gamma {w['gamma']}, s {w['s']}")

    phi0 = uniform_field(shape, w["seed"], mean=w["mean"], amp=0.05)
    prob = chhs.make_problem(shape, 1.0 / n, w["eps"], w["gamma"], w["s"])
    mixed = name.endswith("-mixed")
    cand = ("pre0", "post0", "refine") if mixed else ("pre0", "post0")
    opts = chhs.chhs_default_opts(tol=1e-10, timing=chhs.timing_mask(*cand),
                                  smoother=args.smoother, precision=1 if mixed else 0,
                                  inner_cycles=args.inner_cycles if mixed else 0,
                                  autotune=int(args.autotune))
    sv = chhs.Solver(prob, opts)
    tp = torch.from_numpy(phi0).cuda()
    tc = tp.clone()
    tm = torch.zeros_like(tp)
    tpp = torch.zeros_like(tp)

    sweeps = None
    if args.tune_sweeps:
        # the cycle by time to tolerance on the first step's system, before the
        # warm-up steps, which then run the kept cycle
        sweeps = sv.tune_sweeps(tp, tc, tm, tpp)
        log(f"tuned {SWEEP_KEYS} = {sweeps}")
    sv.timing(reset=True)
    for k in range(args.warmup):
        _, lg = sv.step_log(tp, tc, tm, tpp, 1)
        log(f"warmup step {k + 1}/{args.warmup}: {lg[0][0]['vcycles']} V-cycles, "
            f"res {lg[0][0]['res_norm']:.2e}")
    if copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 device copies of {COPY_BYTES} bytes")
        del src, dst
    torch.cuda.synchronize()
    start_state = [t.cpu().numpy() for t in (tp, tc, tm, tpp)]
    tim_w = sv.timing(reset=True)
    cls = dominant_class(tim_w, cand)
    sv.set_timing(chhs.timing_mask(cls))

    torch.cuda.synchronize()
    with no_gc():
        t0 = time.perf_counter()
        _, lg = sv.step_log(tp, tc, tm, tpp, args.steps)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    tim = sv.timing()
    vcyc = sum(step[0]["vcycles"] for step in lg)
    log(f"timed {args.steps} steps in {elapsed:.3f}s, {vcyc} V-cycles, last res "
        f"{lg[-1][0]['res_norm']:.2e}")

    one3 = " (one red-black step, z marching)" if sv.level_kernels()[0][0] == "zmarch" else " (one color)"
    names = {"pre0": "finest-level pre-smoothing launch" + (
                 " (2 fused red-black steps + residual + restriction)" if dim == 2 else one3),
             "post0": "finest-level post-smoothing launch" + (
                 " (prolongation + 2 fused red-black steps + residual norm)" if dim == 2 else one3),
             "refine": "finest-level FP64 refinement launch"}
    level_kernels = sv.level_kernels()
    kind0 = level_kernels[0][0]
    if cls == "refine":
        bytes_launch = cells * 100 * vcyc / max(1, tim[cls][1])
    else:
        bytes_launch = launch_bytes_per_cell(dim, cls, mixed, kind0) * cells
    traffic = measured_traffic(name, cls, level_kernels[0])
    roofline = roofline_record(cls, tim, bytes_launch, names[cls], traffic)
    for other in cand:
        if other != cls and tim_w[other][1]:
            avg_o = tim_w[other][0] / 1e3 / tim_w[other][1]
            if other == "refine":
                continue
            b_o = launch_bytes_per_cell(dim, other, mixed, kind0) * cells
            roofline.setdefault("other_kernels", {})[other] = {
                "kernel": names[other] + ", timed in the warm-up steps",
                "avg_launch_us": round(avg_o * 1e6, 2),
                "achieved": round(b_o / avg_o / 1e9, 1),
                "algorithmic_bytes_per_launch": b_o,
                "traffic": measured_traffic(name, other, level_kernels[0])}
    kernel_ms = {}
    if breakdown:
        extra = (dict(inner_cycles=args.inner_cycles if mixed else 0) if sweeps is None
                 else dict(zip(SWEEP_KEYS, sweeps)))
        sb = chhs.Solver(prob, chhs.chhs_default_opts(tol=1e-10, timing=1, smoother=args.smoother,
                                                      precision=1 if mixed else 0,
                                                      autotune=int(args.autotune), **extra))
        st_b = [torch.from_numpy(a).cuda() for a in start_state]
        nb = min(args.steps, 5)
        sb.step_log(*st_b, 1)
        sb.timing(reset=True)
        sb.step_log(*st_b, nb)
        kernel_ms = {k: round(v[0] / nb, 4) for k, v in sb.timing().items() if v[1]}
        sb.close()
    sv.close()

    out = {
        "metric": METRIC,
        "value": cells * args.steps / elapsed,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": name, "grid": list(shape), "eps": w["eps"],
                   "gamma": w["gamma"], "s": w["s"], "tol": 1e-10, "cycle": "V(2,2)",
                   "precision": "fp32 inner + fp64 refinement" if mixed else "fp64",
                   **({"inner_cycles": max(1, sweeps[5] if sweeps is not None else args.inner_cycles)}
                      if mixed else {}),
                   "reductions": "mass, E_h, F_h, dissipation every step"},
        "vcycles_per_s": vcyc / elapsed,
        "steps_per_s": args.steps / elapsed,
        "vcycles_per_step": vcyc / args.steps,
        "res_norm_last": lg[-1][0]["res_norm"],
        "kernel_ms_per_step": kernel_ms,
        "level_kernels": [list(k) for k in level_kernels],
        "sweeps": None if sweeps is None else dict(zip(SWEEP_KEYS, sweeps)),
        "roofline": roofline,
        "per_vcycle": None,
    }
    if not mixed and vcyc:
        # HBM fraction of whole V-cycles: the cycle's algorithmic bytes over the
        # wall time per cycle (the per-step setup, copy-out and energies included)
        vb = vcycle_bytes(dim, shape, level_kernels, sweeps)
        t_cyc = elapsed / vcyc
        out["per_vcycle"] = {"algorithmic_bytes": round(vb), "wall_us": round(t_cyc * 1e6, 2),
                             "achieved": round(vb / t_cyc / 1e9, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(vb / t_cyc / 1e9 / HBM_PEAK_GBS, 4)}

    if parity:
        # parity of the same workload at a size the oracle solves in seconds
        from oracle import fas, scheme
        m = 128 if dim == 2 else 32
        sm = (m,) * dim
        prm = scheme.Params(eps=w["eps"], gamma=w["gamma"], s=w["s"], h=1.0 / m)
        ph0 = uniform_field(sm, w["seed"], mean=w["mean"], amp=0.05)
        z = np.zeros(sm)
        ref = fas.solve_step(ph0, ph0, z, z, prm, fas.Opts(tol=1e-10))
        sv2 = chhs.Solver(chhs.make_problem(sm, prm.h, prm.eps, prm.gamma, prm.s),
                          chhs.chhs_default_opts(tol=1e-10, precision=1 if mixed else 0))
        a = torch.from_numpy(ph0).cuda()
        b = a.clone()
        zm, zp = torch.zeros_like(a), torch.zeros_like(a)
        sv2.step(a, b, zm, zp, 1)
        err = float(np.max(np.abs(b.cpu().numpy() - ref.phi)))
        out["parity"] = {"grid": list(sm), "steps": 1, "max_abs_err_phi_vs_oracle": err}
        log(f"parity at {m}^{dim}: max|phi - oracle| = {err:.2e}")
        sv2.close()

    if cpu_baseline:
        log("timing the oracle on a bounded sample (single-threaded NumPy)")
        cpu0 = time.process_time()
        rate, desc, wall = oracle_sample(*start_state, w, vcyc / args.steps)
        cores = max(1, round((time.process_time() - cpu0) / max(wall, 1e-9)))
        out["cpu_baseline"] = {"value": rate, "unit": "cell-updates/s", "cores": cores,
                               "kind": "oracle", "sample": desc, "host": host_info(),
                               "wall_s": round(wall, 2)}
        log(f"oracle: {rate:.3e} cell-updates/s ({wall:.1f}s of CPU work)")
    return out


# ---- counter records --------------------------------------------------------------------

# Finest-level launch classes of the batched workload and how their kernels are
# named; a class's record is taken over its launches that cover every instance
# (the first refinement step of each time step: no instance has converged yet),
# whose counters are the largest of the class.
_CSRC = "paper_1611_02967_amd/csrc/"
# Kernels a counter record covers: (class, dispatch-name pattern, algorithmic
# bytes per cell of one full launch, sources).  Of the dispatches matching a
# smoothing pattern, those with the finest level's workgroup count in the timed
# configuration (the autotuner's other candidates and the coarse levels launch
# other counts), and of those the ones within 2% of the largest FETCH_SIZE and
# WRITE_SIZE (every instance active), are covered; the refinement launch has its
# own task count.
# FP32 tiles: the zero-start pre launch (last template argument true) reads no
# u, 12 B less than the others.
TRAFFIC_KERNELS = [
    ("refine", r"k_mixed_residual_rows", 100.0, ["chhs_refine2d.hip", "chhs_cell.hpp"]),
    ("pre0", r"k_tile2d<float, \w+, 2, 1, false, true, \d+, false, \d+, true>", 46.0,
     ["chhs_tile2d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
    ("pre0", r"k_tile2d<float, \w+, 2, 1, false, true, \d+, false, \d+, false>", 58.0,
     ["chhs_tile2d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
    ("post0", r"k_tile2d<float, \w+, 2, 0, true, true, \d+, false, \d+, false>", 54.0,
     ["chhs_tile2d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
    ("pre0", r"k_stream2d<double, true, 2, 1,", 90.0,
     ["chhs_stream2d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
    ("post0", r"k_stream2d<double, true, 2, 2,", 84.0,
     ["chhs_stream2d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
    # fused 3D step (template arguments T, CORR, TX, TY, PRO, ZERO, L0): pre
    # launches without prolongation; the post class by its first launch, which
    # also reads u_c and ub_c of the coarse parent (6 values per 8 cells); the
    # finest FP64 level (L0) reads no f_phi, f_p
    ("pre0", r"k_step3d<double, false, \d+, \d+, 0, false, true>", 72.0,
     ["chhs_step3d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
    ("post0", r"k_step3d<double, false, \d+, \d+, 1, false, true>", 78.0,
     ["chhs_step3d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
    ("pre0", r"k_step3d<float, true, \d+, \d+, 0, true, false>", 36.0,
     ["chhs_step3d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
    ("pre0", r"k_step3d<float, true, \d+, \d+, 0, false, false>", 48.0,
     ["chhs_step3d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
    ("post0", r"k_step3d<float, true, \d+, \d+, 1, false, false>", 51.0,
     ["chhs_step3d.hip", "chhs_cell.hpp", "chhs_internal.hpp"]),
]


def _counter_rows(path):
    """(dispatch id, kernel name, value, workgroups) of every row of a rocprofv3
    counter collection csv (a file, or the directory rocprofv3 wrote it under)."""
    import csv
    import glob
    files = [path] if os.path.isfile(path) else sorted(
        glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True))
    rows = []
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                wg = int(r.get("Workgroup_Size") or 1)
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]),
                             int(r.get("Grid_Size") or 0) // max(1, wg)))
    return rows


def write_traffic_record(fetch_path, write_path, bench_json):
    """HBM bytes per launch of the dominant finest-level class from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what it reads for the 256 MiB
    device copy of --copy-calibration, into profiles/traffic.json."""
    with open(bench_json) as fh:
        line = [l for l in fh.read().splitlines() if l.startswith("{")][-1]
    run = json.loads(line)
    workload = run["config"]["workload"]
    cfg = run["config"]
    cells = cfg["cells"] if "cells" in cfg else int(math.prod(cfg["grid"]))
    fetch = {d: (k, v) for d, k, v, _ in _counter_rows(fetch_path)}
    write = {d: (k, v) for d, k, v, _ in _counter_rows(write_path)}
    blocks = {d: b for d, _, _, b in _counter_rows(fetch_path)}
    # the smoothing launches of the timed configuration: the finest level's
    # workgroup count (the autotuner's other candidates and the coarse levels
    # launch other counts)
    blocks0 = int(run["level_kernels"][0][2])
    # the calibration copies: device copies whose WRITE_SIZE is the 256 MiB
    # they write (a streaming copy writes every line once; the run's other
    # copies, of the state arrays, have other sizes)
    copies = [d for d, (k, v) in fetch.items() if "copyBuffer" in k and d in write
              and abs(write[d][1] * 1024 - COPY_BYTES) <= 0.05 * COPY_BYTES]
    if not copies:
        raise SystemExit("no 256 MiB copy in the counter runs (run the bench with --copy-calibration)")
    # the largest of the copies' read counts: a repeated copy of the same
    # source can find it in the 256 MB memory-side cache and read almost
    # nothing from HBM
    fk = max(fetch[d][1] for d in copies)
    wk = max(write[d][1] for d in copies)
    read_scale, write_scale = COPY_BYTES / (fk * 1024), COPY_BYTES / (wk * 1024)
    rec = {"workload": workload, "sources": [], "level0_kernel": run["level_kernels"][0],
           "calibration": {"kernel": "device copy of 256 MiB (torch copy_)",
                           "bytes_copied": COPY_BYTES, "fetch_kib": round(fk, 2),
                           "write_kib": round(wk, 2), "read_scale": read_scale,
                           "write_scale": write_scale},
           "launches": {}}
    import re
    for cls, pattern, per_cell, srcs in TRAFFIC_KERNELS:
        ds = sorted(d for d, (k, v) in fetch.items() if re.search(pattern, k)
                    and (cls == "refine" or blocks.get(d) in (blocks0, None, 0)))
        if not ds:
            continue
        # L2 writes back lazily: a dispatch's WRITE_SIZE can miss lines that a
        # later one writes back, so both counters must be within 2% of their
        # largest values
        top = max(fetch[d][1] for d in ds)
        wtop = max(write[d][1] for d in ds if d in write)
        full = [d for d in ds if fetch[d][1] >= 0.98 * top and d in write
                and write[d][1] >= 0.98 * wtop]
        f_sum = sum(fetch[d][1] for d in full)
        w_sum = sum(write[d][1] for d in full)
        counted = f_sum * 1024 * read_scale + w_sum * 1024 * write_scale
        algo = per_cell * cells * len(full)
        ent = rec["launches"].setdefault(cls, {"kernels": [], "dispatches": 0,
                                               "counted_bytes": 0.0, "algorithmic_bytes": 0.0})
        ent["kernels"].append({"pattern": pattern, "dispatches": len(full), "of_dispatches": len(ds),
                               "fetch_kib": round(f_sum / len(full), 2),
                               "write_kib": round(w_sum / len(full), 2),
                               "algorithmic_bytes_per_cell": per_cell})
        ent["dispatches"] += len(full)
        ent["counted_bytes"] += counted
        ent["algorithmic_bytes"] += algo
        rec["sources"] = sorted(set(rec["sources"]) | {_CSRC + f for f in srcs})
    for ent in rec["launches"].values():
        # per launch of the covered mix (the ratio is what the bench applies)
        ent["bytes_per_launch"] = round(ent["counted_bytes"] / ent["dispatches"])
        ent["algorithmic_bytes_per_launch"] = round(ent["algorithmic_bytes"] / ent["dispatches"])
        ent["launches_covered"] = "every instance active (within 2% of the largest counters)"
        del ent["counted_bytes"], ent["algorithmic_bytes"]
    rec["source_sha256"] = kernel_source_hash(rec["sources"])
    try:
        with open(TRAFFIC_FILE) as fh:
            recs = json.load(fh)
    except (OSError, ValueError):
        recs = {}
    recs[workload] = rec
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(recs, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=BATCHED,
                    help=f"{BATCHED} (default) or a single-grid workload name")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-fp64-2048", action="store_true",
                    help="with the batched workload, skip the 2048^2 FP64 extra measurement")
    ap.add_argument("--no-sequential", action="store_true",
                    help="with the batched workload, skip the sequential FP64 loop (and the "
                         "comparisons that need it), e.g. under a counter profiler")
    ap.add_argument("--traffic-record", nargs=3, metavar=("FETCH", "WRITE", "BENCH_JSON"),
                    help="no GPU work: turn two rocprofv3 counter passes of a bench run "
                         "(FETCH_SIZE and WRITE_SIZE, csv output directories) and that run's "
                         "JSON line into the committed traffic record of its workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="before the timed region, copy a 256 MiB device buffer three times "
                         "(the known-size kernel that scales rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="skip the per-class timing pass after the timed region")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="use the default smoothing kernels instead of letting chhs_init time "
                         "the candidates per level and keep the fastest")
    ap.add_argument("--no-tune-sweeps", dest="tune_sweeps", action="store_false",
                    help="keep V(2,2) with piecewise-constant prolongation (and --inner-cycles) "
                         "instead of choosing the sweeps per level, the prolongation and the FP32 "
                         "cycles per refinement by time to tolerance before the warm-up steps")
    ap.add_argument("--inner-cycles", type=int, default=1,
                    help="FP32 correction V-cycles per FP64 refinement (mixed precision)")
    ap.add_argument("--smoother", type=int, default=0,
                    help="0 default (2D strips on the finest level; 3D fused step where segments are long), "
                         "1 2D tiles, 2 2D strips, 3 3D per-cell kernels, 4 3D fused step everywhere")
    args = ap.parse_args()

    if args.traffic_record:
        write_traffic_record(*args.traffic_record)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs one GPU only (--gpus {args.gpus} requested); "
              "the batched and single-grid paths are measured on one MI355X", file=sys.stderr)
        sys.exit(2)

    batched = args.workload == BATCHED
    # the oracle's worker processes are forked before anything touches the GPU
    pool = None
    if batched and not args.no_cpu_baseline:
        pool = make_pool(max(1, min(8, MAX_POOL, os.cpu_count() or 1)))

    import torch

    from paper_1611_02967_amd import build as _build
    if not os.path.exists(_build.LIB):
        log("libchhs.so missing: building")
        _build.build()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"

    try:
        if batched:
            out = run_batched(args, pool)
            if args.copy_calibration:
                src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
                dst = torch.empty_like(src)
                for _ in range(3):
                    dst.copy_(src)
                torch.cuda.synchronize()
                del src, dst
            if not args.no_fp64_2048:
                one = run_single(args, "2d-2048-fp64", cpu_baseline=False, parity=False,
                                 breakdown=False)
                out["fp64_2048"] = {k: one[k] for k in (
                    "value", "unit", "ms_per_step", "steps_per_s", "vcycles_per_step",
                    "vcycles_per_s", "config", "roofline", "per_vcycle", "level_kernels",
                    "sweeps")}
        else:
            out = run_single(args, args.workload, cpu_baseline=not args.no_cpu_baseline,
                             parity=not args.no_parity, breakdown=not args.no_breakdown,
                             copy_calibration=args.copy_calibration)
    finally:
        if pool is not None:
            pool.close()
            pool.join()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
