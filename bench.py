#!/usr/bin/env python
"""Benchmark of the multi-body double-layer solver on one MI355X.

Headline workload (default): 1000 quasi-axisymmetric bodies at seeded
non-overlapping positions in a cube of side 40 -- spheres (r = 0.5), prolate
spheroids (0.5, 0.5, 1.0) and peanuts 0.5 (1 + 0.3 cos 2 psi) in equal
shares, axes bent with curvature ~U[0, 0.3], random rotations, 16 or 32
Gauss-Legendre x 16-32 azimuthal nodes per body (N = 582,592 unknowns,
3.39e11 inter-body pairs per apply), k = 4.

One step = one pass of the whole hot path: node build, self-block assembly
and FP64 factorisation (inverse rounded to FP32 for the mixed path),
mixed-precision solve (FP32 pair sum inside FP64 iterative refinement) to a
relative residual of 1e-6, far field on a 200 x 200 direction grid.

value = inter-body pair interactions evaluated in the timed steps / their wall
time (whole-job throughput; inputs are resident on the device).  Beside it:
time-to-solve at 1e-6 for the mixed and the plain FP64 solver (solve alone
and with assembly + factorisation), their errors against an FP64 solve at
1e-10, the mixed solve with an FP32 factorisation, per-kernel timings (HIP
events on the library stream), the roofline of the dominant kernel, a short
run of the 27-body lattice workload, 32 independent problems solved in one
handle against one handle each, and the CPU oracle timed on the host.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload random_mixed|lattice27]
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic work per inter-body pair and right-hand side: d = y - x (3),
# r^2 (5), 1/r (1), r (1), k r (1), sin + cos (2), (ikr - 1) e^{ikr} (4),
# 1/r^3 (2), n.d (5), scaling (3), complex multiply-add (8)
FLOP_PER_PAIR = 35
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12}

# The paper's own timings, as context (MATLAB on an Intel Xeon server with
# 256 GB of RAM, FP64, dense direct solves except where noted; other
# discretisations and another algorithm, so not a target)
PAPER_CONTEXT = {
    "hardware": "MATLAB, Intel Xeon server, 256 GB RAM, FP64 (the paper's numerical section)",
    "table8_27_bodies_k5": {"N_tot": 69120, "T_ker_s": 97.48, "T_mat_s": 751.03, "T_solve_s": 680.02,
                            "error": 6.61e-12, "solver": "dense direct (mldivide)"},
    "table7_1000_bodies_k5": {"N_tot": 96000, "T_ker_s": 0.57, "T_mat_s": 220.16, "T_solve_s": 307.51,
                              "error": 2.09e-9, "solver": "GMRES with the block-diagonal preconditioner, "
                                                          "identical bodies on a cubic array"},
    "table6_8_bodies_k5": {"N_tot": 102400, "T_ker_s": 273.63, "T_mat_s": 1076.73, "T_solve_s": 2575.58,
                           "error": 5.41e-12, "solver": "dense direct (mldivide)"},
}

WORKLOADS = {
    "random_mixed": ("random_mixed: 1000 bodies (sphere r=0.5 / spheroid (0.5,0.5,1) / peanut "
                     "0.5(1+0.3cos2psi)), kappa~U[0,0.3], cube side 40, 16-32 GL x 16-32 azimuths, "
                     "k=4, mixed solve to 1e-6", 1e-6),
    "lattice27": ("lattice27: 27 bent spheroids (0.5,0.5,1.0), 3x3x3 spacing 3, 32 GL x 64 azimuths, "
                  "N=55296, k=5, mixed solve to 1e-8", 1e-8),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counter_traffic(workload, kind):
    """HBM bytes per launch of the kernel behind timing kind `kind`, from the
    committed FETCH_SIZE / WRITE_SIZE passes of this workload (scaled by the
    copy calibration), or None when they are missing or the kernel's source
    changed since."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", f"{workload}_counters.json")) as f:
            rec = json.load(f)["kernels"][kind]
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
        return rec["fetch_bytes"] + rec["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def far_grid(n=200):
    """n x n directions (theta_i = 2 pi i / n, phi_j = (j + 1/2) pi / n)."""
    th = np.linspace(0, 2 * math.pi, n, endpoint=False)
    ph = (np.arange(n) + 0.5) * math.pi / n
    T, P = np.meshgrid(th, ph, indexing="ij")
    X = np.stack([np.cos(T) * np.sin(P), np.sin(T) * np.sin(P), np.cos(P)], -1)
    return X.reshape(-1, 3)


# ------------------------------------------------------------------ CPU oracle
_W = {}


def _worker_init(workload):
    from oracle import geometry as geo
    from paper_2606_31380_amd import scenarios as sc
    s = sc.WORKLOADS[workload]()
    d = geo.discretize(s)
    rng = np.random.default_rng(0)
    n = d.pos.shape[0]
    _W.update(scen=s, disc=d, mu=rng.standard_normal(n) + 1j * rng.standard_normal(n))


def _worker_pairs(targets):
    """Oracle pair sum on the given target rows (one process, one thread)."""
    from oracle import pairsum as opair
    from threadpoolctl import threadpool_limits
    d, s = _W["disc"], _W["scen"]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        opair.pair_sum(d, s.k, _W["mu"], targets=np.asarray(targets, dtype=np.int64), chunk=16)
        dt = time.perf_counter() - t0
    n = d.pos.shape[0]
    own = np.bincount(d.body, minlength=len(d.bodies))[d.body[np.asarray(targets)]]
    return int(np.sum(n - own)), dt


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload, krylov_applies, budget_s=8.0):
    """The oracle on the host: its pair sum (numpy FP64) on bounded target
    samples of the benchmark workload, one process and one per core; the
    oracle's dense time-to-solve on the two-sphere workload; and the
    time-to-solve of the benchmark workload extrapolated from the all-core
    pair rate (labelled as such, not measured)."""
    from threadpoolctl import threadpool_limits
    from paper_2606_31380_amd import scenarios as sc
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    _worker_init(workload)
    n = _W["disc"].pos.shape[0]
    # one core: calibrate on 32 rows, then a sample of about budget_s / 2
    pairs, dt = _worker_pairs(np.arange(0, 32))
    m1 = int(max(32, min(n, 0.5 * budget_s * 32 / max(dt, 1e-9))))
    tg1 = np.linspace(0, n - 1, m1).astype(np.int64)
    p1, t1 = _worker_pairs(tg1)
    one = {"value": p1 / t1, "unit": "pair-interactions/s", "cores": 1,
           "sample": f"{m1} of {n} target rows ({p1:.3e} pairs, {t1:.1f} s)"}
    log(f"cpu: one core {p1 / t1:.3e} pairs/s")
    # all cores: one process per core on interleaved rows, timed around the map
    per = int(max(8, budget_s * (p1 / t1) / max(1.0, float(n))))
    rows = np.linspace(0, n - 1, per * cores).astype(np.int64)
    chunks = [rows[i::cores] for i in range(cores)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores, initializer=_worker_init, initargs=(workload,)) as pool:
        pool.map(_worker_pairs, [np.arange(4)] * cores)          # warm-up
        t0 = time.perf_counter()
        res = pool.map(_worker_pairs, chunks)
        tall = time.perf_counter() - t0
    pall = sum(r[0] for r in res)
    log(f"cpu: {cores} cores {pall / tall:.3e} pairs/s")
    # dense time-to-solve of the two-sphere workload (setup included)
    from oracle import geometry as geo
    from oracle import solve as osolve
    s1 = sc.two_spheres()
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        d1 = geo.discretize(s1)
        blocks = osolve.self_blocks(d1, s1.k, body_ids=[0])
        blocks[1] = blocks[0]          # the two spheres are congruent
        ta = time.perf_counter()
        b = osolve.rhs_planewave(d1, s1.k, s1.dirs)[:, 0]
        A = osolve.dense_matrix_fast(d1, s1.k, blocks)
        np.linalg.solve(A, b)
        t_cfg1 = time.perf_counter() - t0
    log(f"cpu: two-sphere dense solve {t_cfg1:.1f} s")
    P = _W["scen"].pairs_per_apply()
    rate = pall / tall
    return {"value": rate, "unit": "pair-interactions/s", "cores": cores, "kind": "oracle",
            "sample": f"{rows.size} of {n} target rows of the same workload, {cores} processes "
                      f"({pall:.3e} pairs, {tall:.1f} s, numpy FP64)",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "cores_all": cores,
            "one_core": one,
            "time_to_solve_cfg1_s": t_cfg1,
            "cfg1": {"workload": "two spheres r=0.5 at (+-1,0,0), 16 GL x 32 azimuths, N=1024, k=2, "
                                 "dense LU", "self_block_s": ta - t0, "matrix_and_lu_s": t_cfg1 - (ta - t0),
                     "threads": cores},
            "extrapolated_time_to_solve_s": {
                "value": P * krylov_applies / rate,
                "note": f"NOT MEASURED: {P:.3e} pairs per apply x {krylov_applies} pair sums of the "
                        f"GPU mixed solve / the all-core oracle pair rate"}}


# ------------------------------------------------------------------ GPU runs
def rooflines(ktimes, scen, P, factor_fp64, steps, applies):
    """Per timed kernel kind: algorithmic work per dispatch / average dispatch
    duration.  A pair sum may take several dispatches (its work split into
    launches of bounded workspace): the work per dispatch is then the work of
    the step's pair sums (applies[kind] of P pairs) over its dispatches."""
    # distinct self blocks (equal shape, curvature, discretisation and k)
    bb = scen.bodies
    kb = np.asarray(scen.k)[bb["problem"]]
    keys = {}
    for i in range(len(bb)):
        c = float(bb["c"][i]) if int(bb["shape"][i]) < 3 else 0.0
        key = (int(bb["shape"][i]), float(bb["a"][i]), c, float(bb["kappa"][i]), int(bb["n_panels"][i]),
               int(bb["n_ref"][i]), int(bb["n_theta"][i]), float(kb[i]))
        keys.setdefault(key, i)
    first = np.array(sorted(keys.values()))
    nb_all = scen.nodes_per_body().astype(np.float64)   # every body's block is read per apply
    nb = nb_all[first]
    nth = bb["n_theta"].astype(np.float64)[first]
    npan = (bb["n_panels"] + 2 * bb["n_ref"]).astype(np.float64)[first]
    # mirror-symmetric bodies (sphere, spheroid, peanut, quasi-ellipsoid):
    # the rows s < n_s / 2, j <= N are assembled, (N + 1) / (4 N) of them, and
    # B is inverted through four blocks of orders (n_s / 2)(N +- 1)
    sym = bb["shape"][first] <= 3
    Nh = nth / 2
    rows_frac = np.where(sym, (Nh + 1) / (4 * Nh), 1.0)
    # self-block assembly: per (target row, outer node) the azimuthal modes of
    # the kernel at the minimal grid (L = 128 samples at 35 flop, a 128-point
    # FFT at 5 L log2 L) and the 16 x 2N weighted accumulation (8 flop per
    # term); per (row, panel) one 2N x 2N inverse DFT for 16 functions; outer
    # nodes per row: 2 g on the own panel + g per adjacent panel, with the
    # outer rule's order g = 48 on two or more panels, else 64.  Counted once
    # per distinct block, over the rows assembled.
    per_node = 35 * 128 + 5 * 128 * 7 + 8 * 16 * nth
    per_item = 8 * 16 * nth * nth
    adj = np.where(npan > 1, np.where(npan > 2, 2.0 - 2.0 / npan, 1.0), 0.0)
    g = np.where(npan >= 2, 48.0, 64.0)
    self_flop = float(np.sum(rows_frac * nb * ((2 * g + g * adj) * per_node + (1 + adj) * per_item)))
    # inversion: 8 m^3 per matrix of order m inverted; a trailing update of
    # the 128 columns at k0 is 8 m (m - w) w, w = min(128, m - k0), and the
    # dispatches are one per 128 columns of the largest matrix of each batch
    # (symmetric reduced blocks, other blocks)
    half = npan * 16 / 2
    orders, batches = [], [[], []]
    for i in range(len(nb)):
        ms = [half[i] * (Nh[i] + 1)] * 2 + [half[i] * (Nh[i] - 1)] * 2 if sym[i] else [nb[i]]
        orders += ms
        batches[0 if sym[i] else 1] += ms
    orders = np.array(orders)
    inv_flop = float(np.sum(8.0 * orders ** 3))
    upd_tot = 0.0
    for m in orders:
        for k0 in np.arange(0, m, 128):
            w = min(128.0, m - k0)
            upd_tot += 8.0 * m * (m - w) * w
    upd_disp = sum(int(np.ceil(max(b) / 128)) for b in batches if b)
    upd_flop = float(upd_tot / max(upd_disp, 1))
    # the FP32 block apply is the preconditioner's: when every body is
    # mirror-symmetric it reads the four reduced inverses of each body
    # (sum of their squared orders) instead of the whole block
    h_all = (bb["n_panels"] + 2 * bb["n_ref"]).astype(np.float64) * 8
    N_all = bb["n_theta"].astype(np.float64) / 2
    red_all = 2 * (h_all * (N_all + 1)) ** 2 + 2 * (h_all * (N_all - 1)) ** 2
    f32_apply_elems = float(np.sum(red_all) if np.all(bb["shape"] <= 3) else np.sum(nb_all * nb_all))
    inv_peak = PEAK["fp64"] if factor_fp64 else PEAK["fp32"]
    work = {"pair_sum_fp32": ("alu", FLOP_PER_PAIR * P, PEAK["fp32"], "TFLOP/s"),
            "pair_sum_fp64": ("alu", FLOP_PER_PAIR * P, PEAK["fp64"], "TFLOP/s"),
            "block_apply": ("hbm", float(np.sum(nb_all * nb_all)) * 16.0, PEAK["hbm"], "GB/s"),
            "block_apply_f32": ("hbm", f32_apply_elems * 8.0, PEAK["hbm"], "GB/s"),
            "self_assembly": ("alu", self_flop, PEAK["fp64"], "TFLOP/s"),
            "invert": ("mfma", inv_flop, inv_peak, "TFLOP/s"),
            "invert_update": ("mfma", upd_flop, inv_peak, "TFLOP/s")}
    out = {}
    for name, (cnt, tot) in ktimes.items():
        if cnt == 0 or tot <= 0 or name not in work:
            continue
        bound, units, peak, unit = work[name]
        if name in applies:
            units = units * applies[name] / cnt
        avg_s = tot / cnt / 1e3
        ach = units / avg_s
        scale = 1e9 if unit == "GB/s" else 1e12
        out[name] = {"bound": bound, "achieved": ach / scale, "peak": peak / scale, "unit": unit,
                     "frac": ach / peak, "traffic": counter_traffic(scen.name, name),
                     "avg_launch_ms": avg_s * 1e3, "launches": cnt,
                     "ms_per_step": tot / steps}
    return out


def run_workload(qax, torch, dev, scen, tol, steps, warmup, tune_cache, compare=True):
    stream = torch.cuda.current_stream(dev)
    P = scen.pairs_per_apply()
    h = qax.qax_create(0, stream.cuda_stream)
    xhat = far_grid(200)
    dirs = np.asarray(scen.dirs, dtype=np.float64)
    res = {}
    try:
        qax.qax_build(h, scen.bodies, scen.k)
        N, _ = qax.qax_size(h)
        mu = torch.zeros(N, dtype=torch.complex128, device=dev)
        uinf = torch.zeros(xhat.shape[0], dtype=torch.complex128, device=dev)

        def step(prec):
            qax.qax_build(h, scen.bodies, scen.k)
            qax.qax_assemble_self(h)
            info = qax.qax_solve(h, prec, dirs, mu, 1, tol=tol, maxit=1000)
            qax.qax_farfield(h, mu, xhat, uinf)
            return info

        # launch choices by the library's autotuner (untimed; the geometry of
        # every step is the same, so the choices carry over)
        qax.qax_assemble_self(h)
        t0 = time.perf_counter()
        qax.qax_autotune(h, nrhs_max=1, cache_path=tune_cache)
        res["tuning"] = dict(qax.qax_tuning(h), seconds=time.perf_counter() - t0)
        log(f"{scen.name}: N={N}, autotuned in {res['tuning']['seconds']:.1f} s")
        for _ in range(warmup):
            step(qax.QAX_MIXED)
        log(f"{scen.name}: warm-up done")
        qax.qax_set_timing(h, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for i in range(steps):
            infos.append(step(qax.QAX_MIXED))
            log(f"{scen.name}: step {i + 1}/{steps} iters={infos[-1]['iters']}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ktimes = {name: qax.qax_timing(h, k) for k, name in enumerate(qax.KERNEL_NAMES)}
        qax.qax_set_timing(h, False)
        n32 = sum(i["iters"] for i in infos)          # FP32 pair sums (Krylov steps)
        n64 = sum(i["outer_iters"] for i in infos)     # FP64 true residuals (one per cycle)
        res.update(N=int(N), P=int(P), wall=wall, steps=steps, n32=n32, n64=n64,
                   value=P * (n32 + n64) / wall, ms_per_step=1e3 * wall / steps,
                   kernel_ms_per_step={k: v[1] / steps for k, v in ktimes.items()},
                   rooflines=rooflines(ktimes, scen, P, True, steps,
                                       {"pair_sum_fp32": n32, "pair_sum_fp64": n64}),
                   solver_per_step={"fp32_pair_sums": n32 / steps, "fp64_pair_sums": n64 / steps})
        if not compare:
            return res

        # outside the timed region: precision pattern at 1e-6 and at tol
        def solve(prec, t):
            x = torch.zeros_like(mu)
            i = qax.qax_solve(h, prec, dirs, x, 1, tol=t, maxit=2000)
            return x, i
        ref_tol = 1e-10 if N > 100000 else 1e-12
        ref, iref = solve(qax.QAX_FP64, ref_tol)
        rn = torch.linalg.norm(ref).item()
        log(f"{scen.name}: reference FP64 solve to {ref_tol:g} in {iref['t_solve_s']:.2f} s")

        def err(x):
            return torch.linalg.norm(x - ref).item() / rn
        t_setup = qax.qax_assemble_self(h)
        tts = {"tol": 1e-6, "reference_tol": ref_tol, "setup_s": t_setup,
               "setup_note": "self-block assembly + FP64 factorisation (both solvers use it)"}
        for name, prec in (("mixed", qax.QAX_MIXED), ("fp64", qax.QAX_FP64)):
            x, i = solve(prec, 1e-6)
            tts[name] = {"solve_s": i["t_solve_s"], "with_setup_s": i["t_solve_s"] + t_setup,
                         "err": err(x), "iters": i["iters"], "outer": i["outer_iters"],
                         "rel_res": i["rel_res"]}
            log(f"{scen.name}: {name} 1e-6 in {i['t_solve_s']:.2f} s, err {tts[name]['err']:.2e}")
        # the mixed path with its inverse computed in FP32
        qax.qax_set_factorization(h, qax.QAX_MIXED)
        t_setup32 = qax.qax_assemble_self(h)
        x, i = solve(qax.QAX_MIXED, 1e-6)
        tts["mixed_fp32_factorisation"] = {"setup_s": t_setup32, "solve_s": i["t_solve_s"],
                                           "with_setup_s": i["t_solve_s"] + t_setup32, "err": err(x),
                                           "iters": i["iters"], "outer": i["outer_iters"]}
        qax.qax_set_factorization(h, qax.QAX_FP64)
        qax.qax_assemble_self(h)
        tts["speedup_mixed_vs_fp64"] = tts["fp64"]["solve_s"] / tts["mixed"]["solve_s"]
        tts["speedup_mixed_vs_fp64_with_setup"] = tts["fp64"]["with_setup_s"] / tts["mixed"]["with_setup_s"]
        res["time_to_solve_1e-6"] = tts
        if tol != 1e-6:
            xm, im = solve(qax.QAX_MIXED, tol)
            x6, i6 = solve(qax.QAX_FP64, tol)
            res["time_to_solve_tol"] = {"tol": tol, "mixed_s": im["t_solve_s"], "fp64_s": i6["t_solve_s"],
                                        "mixed_err": err(xm), "fp64_err": err(x6)}
        # pair-sum kernels on their own (HIP events on the library stream)
        qax.qax_set_timing(h, True)
        v = torch.randn(N, dtype=torch.complex128, device=dev)
        o = torch.zeros_like(v)
        for _ in range(3):
            qax.qax_pair_sum(h, qax.QAX_FP64, v, o)
            qax.qax_pair_sum(h, qax.QAX_MIXED, v, o)
        ps64 = qax.qax_timing(h, qax.QAX_K_PAIRSUM_FP64)
        ps32 = qax.qax_timing(h, qax.QAX_K_PAIRSUM_FP32)
        qax.qax_set_timing(h, False)
        res["pair_sum_kernel"] = {
            "fp32_pairs_per_s": P * 3 / (ps32[1] / 1e3), "fp64_pairs_per_s": P * 3 / (ps64[1] / 1e3),
            "fp32_ms_per_apply": ps32[1] / 3, "fp64_ms_per_apply": ps64[1] / 3,
            "fp32_dispatches_per_apply": ps32[0] / 3, "fp64_dispatches_per_apply": ps64[0] / 3}
        # far field on its own
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qax.qax_farfield(h, v, xhat, uinf)
        torch.cuda.synchronize()
        res["farfield_40000_dirs_s"] = time.perf_counter() - t0
    finally:
        qax.qax_destroy(h)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="random_mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 32-problem batched-vs-sequential comparison")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (read if it has this problem, else written)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no "
              "multi-GPU path (sharding by bodies is designed, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_31380_amd import qax
    from paper_2606_31380_amd import scenarios as sc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    desc, tol = WORKLOADS[args.workload]
    scen = sc.WORKLOADS[args.workload]()
    r = run_workload(qax, torch, dev, scen, tol, args.steps, args.warmup, args.tune_cache)
    roofs = r["rooflines"]
    dom = max((k for k in roofs if k != "invert"), key=lambda k: roofs[k]["ms_per_step"])
    roof = {k: v for k, v in roofs[dom].items() if k != "ms_per_step"}
    roof["kernel"] = dom
    out = {
        "metric": "Helmholtz pair-interactions/s + time-to-solve @1e-6 rel err, mixed vs FP64",
        "value": r["value"], "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": desc, "n_unknowns": r["N"], "pairs_per_apply": r["P"]},
        "time_to_solve_1e-6": r["time_to_solve_1e-6"],
        "pair_sum_kernel": r["pair_sum_kernel"],
        "kernel_ms_per_step": r["kernel_ms_per_step"],
        "solver_per_step": r["solver_per_step"],
        "farfield_40000_dirs_s": r["farfield_40000_dirs_s"],
        "roofline": roof,
        "tuning": r["tuning"],
        "kernel_rooflines": roofs,
        "paper_context": PAPER_CONTEXT,
    }
    if "time_to_solve_tol" in r:
        out["time_to_solve_tol"] = r["time_to_solve_tol"]
    if args.workload != "lattice27" and not args.no_secondary:
        s2 = sc.lattice27()
        r2 = run_workload(qax, torch, dev, s2, 1e-8, 5, 1, None)
        out["secondary"] = {"lattice27": {
            "workload": WORKLOADS["lattice27"][0], "pairs_per_s": r2["value"],
            "ms_per_step": r2["ms_per_step"], "steps": 5,
            "time_to_solve_1e-6": r2["time_to_solve_1e-6"], "pair_sum_kernel": r2["pair_sum_kernel"],
            "kernel_ms_per_step": r2["kernel_ms_per_step"],
            "pair_sum_fp32_roofline": r2["rooflines"].get("pair_sum_fp32")}}
    if args.workload != "lattice27" and not args.no_secondary and not args.no_batch:
        # 32 independent problems in one handle against 32 handles one after
        # the other (time to solve to 1e-6); its progress lines go to stderr
        import contextlib
        from paper_2606_31380_amd import batching_bench
        with contextlib.redirect_stdout(sys.stderr):
            out.setdefault("secondary", {})["uneven_batch"] = batching_bench.batch()
    if not args.no_cpu_baseline:
        applies = int(round(r["solver_per_step"]["fp32_pair_sums"] + r["solver_per_step"]["fp64_pair_sums"]))
        out["cpu_baseline"] = cpu_baseline(args.workload, applies)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
