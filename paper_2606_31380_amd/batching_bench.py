"""Measurements of the batching pattern on one GPU (each prints one JSON line):

    python -m paper_2606_31380_amd.batching_bench multi_rhs [--loop-sample 8]
    python -m paper_2606_31380_amd.batching_bench batch
    python -m paper_2606_31380_amd.batching_bench lattice

multi_rhs -- 200 bent spheroids (32 GL x 64 azimuthal nodes, N = 409,600),
k = 6, 64 incident directions: one FP32 / FP64 pair sum over all 64
right-hand sides against 64 single-right-hand-side pair sums; the block apply
of B^-1 with 64 right-hand sides (batched complex GEMM on the matrix cores)
against 64 single-right-hand-side applies; time to solve to 1e-6 with all 64
directions in one lockstep GMRES (independent Krylov spaces sharing each
apply) against one solve per direction (the
per-direction loop is run on the first `--loop-sample` directions and its
total is that time x 64 / sample, stated as such), and by block GMRES (one
Krylov space shared by the 64 directions).

batch -- 32 independent problems (1-100 bent spheroids each, 16-32 GL x
16-64 azimuthal nodes per body, own k in [1, 10], one direction each,
N = 1,746,400 in total): one handle holding all problems (one launch per
kernel for all of them, captured GMRES steps) against 32 handles solved one
after the other; time to solve to 1e-6 (mixed and FP64) and set-up time.

lattice -- regular 10 x 10 x 10 arrays of identical bent spheroids (the
block-reuse configuration of Example 4: 96 nodes per body, and 512 nodes per
body), k = 2: the direct pair sum against the block-Toeplitz apply
(qax_lattice), 1 and 16 right-hand sides, FP64 and FP32 tables, the
per-frequency product's share and bandwidth, and the time to solve to 1e-6.

Inputs are synthetic and seeded (paper_2606_31380_amd.scenarios).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _sync():
    import torch
    torch.cuda.synchronize()


def _timed(fn):
    _sync()
    t0 = time.perf_counter()
    out = fn()
    _sync()
    return time.perf_counter() - t0, out


def multi_rhs(loop_sample: int) -> dict:
    import torch

    from paper_2606_31380_amd import qax
    from paper_2606_31380_amd import scenarios as sc

    dev = torch.device("cuda", 0)
    s = sc.lattice_like_random()
    nrhs = s.dirs.shape[0]
    P = s.pairs_per_apply()
    res = {"workload": "200 bent spheroids (0.5, 0.5, 1.0), 32 GL x 64 azimuths, N = 409,600, "
                       "k = 6, 64 directions", "pairs_per_apply": int(P), "nrhs": nrhs}
    print("multi_rhs: building", flush=True)
    with qax.Problem(s) as Pr:
        t_setup, _ = _timed(lambda: qax.qax_assemble_self(Pr.h))
        res["setup_assemble_invert_s"] = t_setup
        qax.qax_autotune(Pr.h, nrhs_max=nrhs)
        res["tuning"] = qax.qax_tuning(Pr.h)
        print(f"multi_rhs: assembled in {t_setup:.2f} s, tuned", flush=True)
        N = Pr.N
        g = torch.Generator(device="cpu").manual_seed(0)
        V = torch.randn(N * nrhs, dtype=torch.complex128, generator=g).to(dev)
        O = torch.zeros_like(V)
        v1 = torch.zeros(N, dtype=torch.complex128, device=dev)
        o1 = torch.zeros_like(v1)
        Vm = V.view(N, nrhs)
        for prec, name in ((qax.QAX_MIXED, "fp32"), (qax.QAX_FP64, "fp64")):
            qax.qax_pair_sum(Pr.h, prec, V, O, nrhs)                       # warm-up
            tb, _ = _timed(lambda: qax.qax_pair_sum(Pr.h, prec, V, O, nrhs))

            def loop():
                for r in range(nrhs):
                    v1.copy_(Vm[:, r])
                    qax.qax_pair_sum(Pr.h, prec, v1, o1, 1)
            tl, _ = _timed(loop)
            res[f"pair_sum_{name}"] = {"block_s": tb, "per_rhs_loop_s": tl, "speedup": tl / tb,
                                       "block_pairs_rhs_per_s": P * nrhs / tb}
            qax.qax_block_apply(Pr.h, 1, prec, V, O, nrhs)
            tb, _ = _timed(lambda: qax.qax_block_apply(Pr.h, 1, prec, V, O, nrhs))

            def loop_apply():
                for r in range(nrhs):
                    v1.copy_(Vm[:, r])
                    qax.qax_block_apply(Pr.h, 1, prec, v1, o1, 1)
            tl, _ = _timed(loop_apply)
            res[f"block_apply_inverse_{name}"] = {"block_gemm_s": tb, "per_rhs_loop_s": tl,
                                                  "speedup": tl / tb}
            print(f"multi_rhs: {name} applies done", flush=True)
        # time to solve, all directions in lockstep (independent Krylov
        # spaces sharing the applies), then by block GMRES (one shared space)
        X = torch.zeros(N * nrhs, dtype=torch.complex128, device=dev)
        info = qax.qax_solve(Pr.h, qax.QAX_MIXED, s.dirs, X, nrhs, tol=1e-6, maxit=400)
        res["solve_lockstep_mixed"] = {"s": info["t_solve_s"], "iters": info["iters"],
                                       "outer_iters": info["outer_iters"], "rel_res": info["rel_res"]}
        print(f"multi_rhs: lockstep solve {info['t_solve_s']:.2f} s", flush=True)
        qax.qax_set_solver(Pr.h, qax.QAX_SOLVER_BLOCK)
        Xb = torch.zeros_like(X)
        ib = qax.qax_solve(Pr.h, qax.QAX_MIXED, s.dirs, Xb, nrhs, tol=1e-6, maxit=400)
        qax.qax_set_solver(Pr.h, qax.QAX_SOLVER_LOCKSTEP)
        res["solve_block_gmres_mixed"] = {"s": ib["t_solve_s"], "iters": ib["iters"],
                                          "outer_iters": ib["outer_iters"], "rel_res": ib["rel_res"],
                                          "rel_diff_to_lockstep": (torch.linalg.norm(Xb - X)
                                                                   / torch.linalg.norm(X)).item()}
        print(f"multi_rhs: block GMRES solve {ib['t_solve_s']:.2f} s", flush=True)
        # one solve per direction, on a sample of the directions
        ts, its = 0.0, []
        x1 = torch.zeros(N, dtype=torch.complex128, device=dev)
        for r in range(loop_sample):
            inf = qax.qax_solve(Pr.h, qax.QAX_MIXED, s.dirs[r:r + 1], x1, 1, tol=1e-6, maxit=400)
            ts += inf["t_solve_s"]
            its.append(inf["iters"])
            # the lockstep solution of this direction agrees with its own solve
            if r == 0:
                xb = X.view(N, nrhs)[:, 0]
                res["block_vs_single_first_direction_rel_diff"] = (
                    torch.linalg.norm(xb - x1) / torch.linalg.norm(x1)).item()
        res["solve_per_rhs_loop_mixed"] = {"sample": loop_sample, "sample_s": ts,
                                           "estimated_total_s": ts * nrhs / loop_sample,
                                           "iters": its}
        res["solve_speedup_lockstep_vs_loop"] = ts * nrhs / loop_sample / info["t_solve_s"]
        res["solve_speedup_block_gmres_vs_loop"] = ts * nrhs / loop_sample / ib["t_solve_s"]
        print("multi_rhs: per-direction solves done", flush=True)
    return res


def batch() -> dict:
    import torch

    from paper_2606_31380_amd import qax
    from paper_2606_31380_amd import scenarios as sc

    dev = torch.device("cuda", 0)
    s = sc.uneven_batch()
    npb = s.bodies["problem"]
    dirs = s.notes["dirs"]
    res = {"workload": "32 independent problems, 1-100 bent spheroids each, 16-32 GL x 16-64 "
                       "azimuths per body, k in [1, 10], one direction each",
           "n_unknowns": int(s.nodes_per_body().sum()), "pairs_per_apply": int(s.pairs_per_apply())}
    print(f"batch: {len(s.bodies)} bodies, N = {res['n_unknowns']}", flush=True)
    with qax.Problem(s) as Pr:
        t_setup, _ = _timed(lambda: qax.qax_assemble_self(Pr.h))
        qax.qax_autotune(Pr.h, nrhs_max=1)
        print(f"batch: batched set-up {t_setup:.2f} s", flush=True)
        out = {"setup_s": t_setup}
        for prec, name in ((qax.QAX_MIXED, "mixed"), (qax.QAX_FP64, "fp64")):
            x = torch.zeros(Pr.N, dtype=torch.complex128, device=dev)
            info = qax.qax_solve(Pr.h, prec, dirs, x, 1, tol=1e-6, maxit=400)
            out[name] = {"s": info["t_solve_s"], "iters": info["iters"],
                         "outer_iters": info["outer_iters"], "rel_res": info["rel_res"]}
            print(f"batch: batched {name} solve {info['t_solve_s']:.2f} s", flush=True)
            if name == "mixed":
                xb = x.cpu().numpy()
        res["batched"] = out
        offsets = Pr.offsets
    seq = {"setup_s": 0.0, "mixed": {"s": 0.0, "iters": []}, "fp64": {"s": 0.0, "iters": []}}
    worst = 0.0
    for p in range(len(s.k)):
        rows = s.bodies[npb == p].copy()
        rows["problem"] = 0
        sp = sc.Scenario(f"p{p}", rows, np.array([s.k[p]]), dirs[p:p + 1])
        with qax.Problem(sp) as Pp:
            t, _ = _timed(lambda: qax.qax_assemble_self(Pp.h))
            seq["setup_s"] += t
            for prec, name in ((qax.QAX_MIXED, "mixed"), (qax.QAX_FP64, "fp64")):
                x = torch.zeros(Pp.N, dtype=torch.complex128, device=dev)
                info = qax.qax_solve(Pp.h, prec, dirs[p:p + 1], x, 1, tol=1e-6, maxit=400)
                seq[name]["s"] += info["t_solve_s"]
                seq[name]["iters"].append(info["iters"])
                if name == "mixed":
                    b0 = int(np.nonzero(npb == p)[0][0])
                    b1 = int(np.nonzero(npb == p)[0][-1]) + 1
                    seg = xb[offsets[b0]:offsets[b1]]
                    xs = x.cpu().numpy()
                    worst = max(worst, float(np.linalg.norm(seg - xs) / np.linalg.norm(xs)))
        print(f"batch: sequential problem {p} done", flush=True)
    res["sequential"] = seq
    res["batched_vs_sequential_max_rel_diff_mixed"] = worst
    res["solve_speedup_batched_vs_sequential"] = {
        "mixed": seq["mixed"]["s"] / res["batched"]["mixed"]["s"],
        "fp64": seq["fp64"]["s"] / res["batched"]["fp64"]["s"]}
    return res


def lattice() -> dict:
    """Regular cubic arrays of identical bent spheroids (Example 4's block
    reuse configuration): direct pair sum against the block-Toeplitz apply."""
    import torch

    from paper_2606_31380_amd import qax
    from paper_2606_31380_amd import scenarios as sc

    dev = torch.device("cuda", 0)
    out = []
    for n_panels, n_theta in ((1, 6), (2, 16)):
        s = sc.cubic_array(10, n_panels=n_panels, n_theta=n_theta, k=2.0)
        rec = {"workload": f"10x10x10 identical bent spheroids (0.5, 0.5, 1.0), kappa 0.2, spacing 3, "
                           f"{16 * n_panels} GL x {n_theta} azimuths, k = 2",
               "pairs_per_apply": int(s.pairs_per_apply())}
        with qax.Problem(s) as Pr:
            N = Pr.N
            rec["n_unknowns"] = N
            nb = N // 1000
            t_asm, _ = _timed(lambda: qax.qax_assemble_self(Pr.h))
            rec["setup_assemble_invert_s"] = t_asm
            g = torch.Generator(device="cpu").manual_seed(0)
            for nrhs in (1, 16):
                V = torch.randn(N * nrhs, dtype=torch.complex128, generator=g).to(dev)
                O = torch.zeros_like(V)
                for prec, name in ((qax.QAX_FP64, "fp64"), (qax.QAX_MIXED, "fp32")):
                    qax.qax_pair_sum(Pr.h, prec, V, O, nrhs)
                    t, _ = _timed(lambda: qax.qax_pair_sum(Pr.h, prec, V, O, nrhs))
                    rec[f"direct_pair_sum_{name}_nrhs{nrhs}_s"] = t
            solve = n_panels == 1      # the direct solve of the finer array takes minutes
            if solve:
                x = torch.zeros(N, dtype=torch.complex128, device=dev)
                info = qax.qax_solve(Pr.h, qax.QAX_MIXED, s.dirs, x, 1, tol=1e-6, maxit=3000)
                rec["direct_solve_mixed_1e-6"] = {"s": info["t_solve_s"], "iters": info["iters"]}
            print(f"lattice {nb}: direct done", flush=True)
            t_lat, _ = _timed(lambda: qax.qax_lattice(Pr.h))
            rec["lattice_setup_s"] = t_lat
            F = 19 ** 3
            rec["frequencies"] = F
            for nrhs in (1, 16):
                V = torch.randn(N * nrhs, dtype=torch.complex128, generator=g).to(dev)
                O = torch.zeros_like(V)
                for prec, name, kind, eb in ((qax.QAX_FP64, "fp64", qax.QAX_K_LATTICE_F64, 16),
                                             (qax.QAX_MIXED, "fp32", qax.QAX_K_LATTICE_F32, 8)):
                    qax.qax_pair_sum(Pr.h, prec, V, O, nrhs)
                    reps = 20
                    t, _ = _timed(lambda: [qax.qax_pair_sum(Pr.h, prec, V, O, nrhs) for _ in range(reps)])
                    qax.qax_set_timing(Pr.h, True)
                    for _ in range(reps):
                        qax.qax_pair_sum(Pr.h, prec, V, O, nrhs)
                    cnt, tot = qax.qax_timing(Pr.h, kind)
                    qax.qax_set_timing(Pr.h, False)
                    prod_ms = tot / max(cnt, 1)
                    table_bytes = F * nb * nb * eb
                    r = {"apply_s": t / reps, "product_ms": prod_ms,
                         "speedup_vs_direct": rec[f"direct_pair_sum_{name}_nrhs{nrhs}_s"] / (t / reps)}
                    if nrhs == 1:
                        r["product_table_GBps"] = table_bytes / (prod_ms * 1e-3) / 1e9
                        r["product_hbm_frac"] = r["product_table_GBps"] / 8000.0
                    else:
                        flop = 8.0 * F * nb * nb * nrhs
                        r["product_TFLOPs"] = flop / (prod_ms * 1e-3) / 1e12
                    rec[f"lattice_{name}_nrhs{nrhs}"] = r
            x2 = torch.zeros(N, dtype=torch.complex128, device=dev)
            info = qax.qax_solve(Pr.h, qax.QAX_MIXED, s.dirs, x2, 1, tol=1e-6, maxit=3000)
            rec["lattice_solve_mixed_1e-6"] = {"s": info["t_solve_s"], "iters": info["iters"]}
            if solve:
                rec["solve_speedup"] = rec["direct_solve_mixed_1e-6"]["s"] / info["t_solve_s"]
                rec["solution_rel_diff"] = (torch.linalg.norm(x2 - x) / torch.linalg.norm(x)).item()
            print(f"lattice {nb}: lattice done", flush=True)
        out.append(rec)
    return {"arrays": out}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["multi_rhs", "batch", "lattice"])
    ap.add_argument("--loop-sample", type=int, default=8)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if args.which == "multi_rhs":
        r = multi_rhs(args.loop_sample)
    elif args.which == "batch":
        r = batch()
    else:
        r = lattice()
    r["measurement"] = args.which
    print(json.dumps(r))
    return 0


if __name__ == "__main__":
    sys.exit(main())
