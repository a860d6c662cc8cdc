#!/usr/bin/env python
"""Benchmark of the multi-body double-layer solver on one MI355X.

One step = one pass of the whole hot path over the 27-body lattice workload
(27 bent prolate spheroids, 32 GL x 64 azimuthal nodes each, 55,296 unknowns,
k = 5, paper incident direction): node build, self-block assembly and
inversion, mixed-precision solve (FP32 pair sum inside FP64 iterative
refinement) to a relative residual of 1e-8, far field on the 200 x 200 grid.

value = inter-body pair interactions evaluated in the timed steps / their wall
time (whole-job throughput; inputs are resident on the device).  The FP64
solve, the achieved error against an FP64 reference, per-kernel timings
(HIP events on the library stream), the roofline of the dominant kernel and
the CPU oracle's pair rate on a bounded sample are reported beside it.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
from __future__ import annotations

import argparse
import json
import math
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


COUNTERS = os.path.join(ROOT, "profiles", "lattice27_counters.json")


def counter_traffic(kind):
    """HBM bytes per launch of the kernel behind timing kind `kind`, from the
    committed FETCH_SIZE / WRITE_SIZE passes (scaled by the copy calibration),
    or None when they are missing or the kernel's source changed since."""
    import hashlib
    try:
        with open(COUNTERS) as f:
            rec = json.load(f)["kernels"][kind]
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
        return rec["fetch_bytes"] + rec["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def far_grid(n=200):
    th = np.linspace(0, 2 * math.pi, n, endpoint=False)
    ph = (np.arange(n) + 0.5) * math.pi / n
    T, P = np.meshgrid(th, ph, indexing="ij")
    X = np.stack([np.cos(T) * np.sin(P), np.sin(T) * np.sin(P), np.cos(P)], -1)
    # (theta_i, phi_j) with j >= n/2 is the antipode of (theta_{i+n/2}, phi_{n-1-j}):
    # stored as its exact negation (the same point up to rounding), so the far
    # field can evaluate the pair with one phase
    h = n // 2
    X[:, h:] = -X[(np.arange(n) + h) % n][:, h - 1::-1]
    return X.reshape(-1, 3)


def cpu_baseline(scen, budget_s=12.0):
    """The oracle's pair sum, timed on the host on a bounded target sample
    (one thread: numpy/BLAS pools limited to 1)."""
    from oracle import geometry as geo
    from oracle import pairsum as opair
    d = geo.discretize(scen)
    n = d.pos.shape[0]
    rng = np.random.default_rng(0)
    mu = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        tg = np.arange(0, 64)
        t0 = time.perf_counter()
        opair.pair_sum(d, scen.k, mu, targets=tg)
        dt = time.perf_counter() - t0
        per_target = dt / tg.shape[0]
        m = int(max(64, min(n, budget_s / max(per_target, 1e-9))))
        tg = np.linspace(0, n - 1, m).astype(np.int64)
        t0 = time.perf_counter()
        opair.pair_sum(d, scen.k, mu, targets=tg)
        dt = time.perf_counter() - t0
    own = np.bincount(d.body, minlength=len(d.bodies))[d.body[tg]]
    pairs = int(np.sum(n - own))
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"{m} of {n} target rows of the same workload ({pairs:.3e} pairs, {dt:.1f} s, numpy FP64, 1 thread)"}


def artificial_solution_error(qax, h, scen, N, dev):
    """Relative error of the near and far field recovered from the boundary
    values of point sources inside the bodies (FP64 solve at 1e-12, mixed at
    1e-8), on 200 points of a shell around the bodies."""
    import torch
    k = float(scen.k[0])
    pos = torch.zeros(N * 3, dtype=torch.float64, device=dev)
    aw = torch.zeros_like(pos)
    qax.qax_nodes(h, pos, aw)
    y = pos.cpu().numpy().reshape(-1, 3)
    cen = np.stack([scen.bodies["cx"], scen.bodies["cy"], scen.bodies["cz"]], 1)
    z = cen + np.array([0.04, -0.03, 0.08])

    def field(x):
        r = np.linalg.norm(x[:, None, :] - z[None, :, :], axis=2)
        return (np.exp(1j * k * r) / (4 * math.pi * r)).sum(axis=1)
    b = torch.from_numpy(field(y)).to(dev)
    c = cen.mean(axis=0)
    rng = np.random.default_rng(7)
    u = rng.standard_normal((200, 3))
    xhat = u / np.linalg.norm(u, axis=1)[:, None]
    pts = c + xhat * (np.abs(cen - c).max() + 6.0)
    exact = field(pts)
    ff_exact = np.exp(-1j * k * (xhat @ z.T)).sum(axis=1) / (4 * math.pi)
    out = {}
    for prec, tol, name in ((qax.QAX_FP64, 1e-12, "fp64"), (qax.QAX_MIXED, 1e-8, "mixed")):
        mu = torch.zeros(N, dtype=torch.complex128, device=dev)
        qax.qax_solve_rhs(h, prec, b, mu, 1, tol=tol, maxit=1000)
        un = torch.zeros(pts.shape[0], dtype=torch.complex128, device=dev)
        qax.qax_nearfield(h, mu, pts, un)
        ff = torch.zeros(pts.shape[0], dtype=torch.complex128, device=dev)
        qax.qax_farfield(h, mu, xhat, ff)
        out[name] = {"tol": tol,
                     "near_rel_err": float(np.linalg.norm(un.cpu().numpy() - exact) / np.linalg.norm(exact)),
                     "far_rel_err": float(np.linalg.norm(ff.cpu().numpy() - ff_exact) / np.linalg.norm(ff_exact))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (read if it has this problem, else written)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_31380_amd import qax
    from paper_2606_31380_amd import scenarios as sc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    scen = sc.lattice27()
    P = scen.pairs_per_apply()
    h = qax.qax_create(0, stream.cuda_stream)
    xhat = far_grid(200)
    dirs = np.asarray(scen.dirs, dtype=np.float64)

    qax.qax_build(h, scen.bodies, scen.k)
    N, _ = qax.qax_size(h)
    mu = torch.zeros(N, dtype=torch.complex128, device=dev)
    uinf = torch.zeros(xhat.shape[0], dtype=torch.complex128, device=dev)

    def step(prec):
        qax.qax_build(h, scen.bodies, scen.k)
        qax.qax_assemble_self(h)
        info = qax.qax_solve(h, prec, dirs, mu, 1, tol=args.tol, maxit=1000)
        qax.qax_farfield(h, mu, xhat, uinf)
        return info

    # launch choices by the library's autotuner (untimed; the geometry of
    # every step is the same, so the choices carry over)
    qax.qax_assemble_self(h)
    qax.qax_autotune(h, nrhs_max=1, cache_path=args.tune_cache)
    tuning = qax.qax_tuning(h)
    for _ in range(args.warmup):
        step(qax.QAX_MIXED)
    qax.qax_set_timing(h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step(qax.QAX_MIXED) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ktimes = {name: qax.qax_timing(h, k) for k, name in enumerate(qax.KERNEL_NAMES)}
    qax.qax_set_timing(h, False)

    n32 = sum(i["iters"] for i in infos)          # FP32 pair sums (Krylov steps)
    n64 = sum(i["outer_iters"] for i in infos)     # FP64 pair sums (true residuals)
    pairs = P * (n32 + n64)
    value = pairs / wall
    ms_per_step = 1e3 * wall / args.steps

    # comparison outside the timed region: FP64 and mixed time-to-solve, error
    ref = torch.zeros_like(mu)
    qax.qax_solve(h, qax.QAX_FP64, dirs, ref, 1, tol=1e-12, maxit=2000)
    x64 = torch.zeros_like(mu)
    i64 = qax.qax_solve(h, qax.QAX_FP64, dirs, x64, 1, tol=args.tol, maxit=1000)
    xm = torch.zeros_like(mu)
    im = qax.qax_solve(h, qax.QAX_MIXED, dirs, xm, 1, tol=args.tol, maxit=1000)
    err64 = (torch.linalg.norm(x64 - ref) / torch.linalg.norm(ref)).item()
    errm = (torch.linalg.norm(xm - ref) / torch.linalg.norm(ref)).item()
    # time-to-solve at the 1e-6 error level
    x6m = torch.zeros_like(mu)
    i6m = qax.qax_solve(h, qax.QAX_MIXED, dirs, x6m, 1, tol=1e-6, maxit=1000)
    x66 = torch.zeros_like(mu)
    i66 = qax.qax_solve(h, qax.QAX_FP64, dirs, x66, 1, tol=1e-6, maxit=1000)
    e6m = (torch.linalg.norm(x6m - ref) / torch.linalg.norm(ref)).item()
    e66 = (torch.linalg.norm(x66 - ref) / torch.linalg.norm(ref)).item()
    # pair-sum kernel rates on their own (HIP events on the library stream)
    qax.qax_set_timing(h, True)
    v = torch.randn(N, dtype=torch.complex128, device=dev)
    o = torch.zeros_like(v)
    for _ in range(5):
        qax.qax_pair_sum(h, qax.QAX_FP64, v, o)
        qax.qax_pair_sum(h, qax.QAX_MIXED, v, o)
    ps64 = qax.qax_timing(h, qax.QAX_K_PAIRSUM_FP64)
    ps32 = qax.qax_timing(h, qax.QAX_K_PAIRSUM_FP32)
    qax.qax_set_timing(h, False)
    # accuracy against an exact solution: boundary values of point sources
    # inside the bodies, the solved density's field on a shell around them
    art = artificial_solution_error(qax, h, scen, N, dev)
    # near-field throughput on a 200 x 200 grid of points on a shell
    pts = 10.0 * far_grid(200)
    un = torch.zeros(pts.shape[0], dtype=torch.complex128, device=dev)
    qax.qax_nearfield(h, v, pts, un)
    torch.cuda.synchronize()
    t0n = time.perf_counter()
    qax.qax_nearfield(h, v, pts, un)
    torch.cuda.synchronize()
    t_near = time.perf_counter() - t0n

    # rooflines of the timed kernels; "roofline" is the dominant one
    nb = scen.nodes_per_body().astype(np.float64)
    nth = scen.bodies["n_theta"].astype(np.float64)
    npan = scen.bodies["n_panels"].astype(np.float64)
    # self-block assembly: per (target row, outer node) the azimuthal modes of
    # the kernel at the minimal grid (L = 128 samples at 35 flop, a 128-point
    # FFT at 5 L log2 L) and the 16 x 2N weighted accumulation (8 flop per
    # term); per (row, panel) one 2N x 2N inverse DFT for 16 functions; outer
    # nodes per row: 2 g on the own panel + g per adjacent panel, with the
    # outer rule's order g = 48 on two or more panels, else 64
    per_node = 35 * 128 + 5 * 128 * 7 + 8 * 16 * nth
    per_item = 8 * 16 * nth * nth
    adj = np.where(npan > 1, np.where(npan > 2, 2.0 - 2.0 / npan, 1.0), 0.0)
    g = np.where(npan >= 2, 48.0, 64.0)
    self_flop = float(np.sum(nb * ((2 * g + g * adj) * per_node + (1 + adj) * per_item)))
    # the inversion of the mixed path runs in FP32 (matrix cores at the FP32 rate)
    inv_flop = float(np.sum(8.0 * nb ** 3))
    # one trailing update of the inversion: rank-128 complex update of every
    # block (128-column panels)
    upd_flop = float(np.sum(8.0 * nb * nb * 128))
    work = {"pair_sum_fp32": ("alu", FLOP_PER_PAIR * P, PEAK["fp32"], "TFLOP/s"),
            "pair_sum_fp64": ("alu", FLOP_PER_PAIR * P, PEAK["fp64"], "TFLOP/s"),
            "block_apply": ("hbm", float(np.sum(nb * nb)) * 16.0, PEAK["hbm"], "GB/s"),
            "block_apply_f32": ("hbm", float(np.sum(nb * nb)) * 8.0, PEAK["hbm"], "GB/s"),
            "self_assembly": ("alu", self_flop, PEAK["fp64"], "TFLOP/s"),
            "invert": ("mfma", inv_flop, PEAK["fp32"], "TFLOP/s"),
            "invert_update": ("mfma", upd_flop, PEAK["fp32"], "TFLOP/s")}
    rooflines = {}
    for name, (cnt, tot) in ktimes.items():
        if cnt == 0 or tot <= 0:
            continue
        bound, units, peak, unit = work[name]
        avg_s = tot / cnt / 1e3
        ach = units / avg_s
        scale = 1e9 if unit == "GB/s" else 1e12
        rooflines[name] = {"bound": bound, "achieved": ach / scale, "peak": peak / scale,
                           "unit": unit, "frac": ach / peak, "traffic": counter_traffic(name),
                           "avg_launch_ms": avg_s * 1e3, "launches": cnt}
    # dominant single kernel by time per step ("invert" spans several kernels)
    dom = max((k for k in ktimes if k != "invert"), key=lambda k: ktimes[k][1])
    roof = dict(rooflines[dom], kernel=dom)
    if dom == "pair_sum_fp32":
        # packed FP32 instructions are disabled in this build: one FP32 FMA per
        # lane and cycle, 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
        roof["peak_without_packed_fp32"] = PEAK["fp32"] / 2 / 1e12
        roof["frac_without_packed_fp32"] = roof["achieved"] / roof["peak_without_packed_fp32"]

    out = {
        "metric": "Helmholtz pair-interactions/s + time-to-solve @1e-6 rel err, mixed vs FP64",
        "value": value, "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "lattice27: 27 bent spheroids (0.5,0.5,1.0), 3x3x3 spacing 3, "
                               "32 GL x 64 azimuths, N=55296, k=5, mixed solve to 1e-8",
                   "n_unknowns": int(N), "pairs_per_apply": int(P)},
        "time_to_solve_1e-6": {"mixed_s": i6m["t_solve_s"], "fp64_s": i66["t_solve_s"],
                               "mixed_err": e6m, "fp64_err": e66,
                               "mixed_iters": i6m["iters"], "fp64_iters": i66["iters"]},
        "time_to_solve_tol": {"tol": args.tol, "mixed_s": im["t_solve_s"], "fp64_s": i64["t_solve_s"],
                              "mixed_err": errm, "fp64_err": err64},
        "pair_sum_kernel": {
            "fp32_pairs_per_s": P * ps32[0] / (ps32[1] / 1e3) if ps32[1] > 0 else None,
            "fp64_pairs_per_s": P * ps64[0] / (ps64[1] / 1e3) if ps64[1] > 0 else None,
            "fp32_ms": ps32[1] / max(ps32[0], 1), "fp64_ms": ps64[1] / max(ps64[0], 1)},
        "kernel_ms_per_step": {k: v[1] / args.steps for k, v in ktimes.items()},
        "artificial_solution": art,
        "nearfield_40000_points": {"s": t_near, "point_source_pairs_per_s": pts.shape[0] * N / t_near},
        "solver_iters_per_step": {"fp32_pair_sums": n32 / args.steps, "fp64_pair_sums": n64 / args.steps},
        "roofline": roof,
        "tuning": tuning,
        "kernel_rooflines": rooflines,
    }
    qax.qax_destroy(h)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scen)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
