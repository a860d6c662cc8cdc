"""Fixed sequence of library calls on one benchmark workload (the 1000-body
workload by default, or the 27-body lattice), for hardware-counter and
kernel-trace runs under rocprofv3:

    rocprofv3 --pmc FETCH_SIZE -d out -- python3 -m paper_2606_31380_amd.profile_workload [tune_cache [workload]]

It first runs one plain elementwise kernel of known traffic (y = 2 x over
2^27 doubles: 1 GiB read, 1 GiB written) so that the memory counters can be
scaled, then: node build, self-block assembly and inversion, the autotuner
(as bench.py runs it; with a cache file written by `bench.py --tune-cache`
the launch choices are those of the benchmark, not re-timed under the
profiler), one FP64 and one FP32 pair sum, block applies (B and B^-1 in FP64,
B^-1 in FP32; one and eight right-hand sides), one eight-column FP32 pair sum
and the far field on the 200 x 200 direction grid.  Every step prints a line.
"""
from __future__ import annotations

import math
import sys

import numpy as np


def main(tune_cache=None, workload="random_mixed") -> int:
    import torch

    from paper_2606_31380_amd import qax
    from paper_2606_31380_amd import scenarios as sc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n_copy = 1 << 27
    x = torch.ones(n_copy, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    print(f"copy calibration: {n_copy * 8} bytes read, {n_copy * 8} bytes written", flush=True)
    del x, y

    scen = sc.WORKLOADS[workload]()
    h = qax.qax_create(0, torch.cuda.current_stream(dev).cuda_stream)
    try:
        qax.qax_build(h, scen.bodies, scen.k)
        N, _ = qax.qax_size(h)
        print(f"build: N = {N}", flush=True)
        qax.qax_assemble_self(h)
        print("assemble_self (assembly + inversion)", flush=True)
        qax.qax_autotune(h, nrhs_max=1, cache_path=tune_cache)
        print(f"autotune: {qax.qax_tuning(h)}", flush=True)
        g = torch.Generator(device="cpu").manual_seed(0)
        v1 = torch.randn(N, dtype=torch.complex128, generator=g).to(dev)
        o1 = torch.zeros_like(v1)
        qax.qax_pair_sum(h, qax.QAX_FP64, v1, o1)
        qax.qax_pair_sum(h, qax.QAX_MIXED, v1, o1)
        torch.cuda.synchronize()
        print("pair sums: FP64, FP32 (one right-hand side)", flush=True)
        qax.qax_block_apply(h, 0, qax.QAX_FP64, v1, o1, 1)
        qax.qax_block_apply(h, 1, qax.QAX_FP64, v1, o1, 1)
        qax.qax_block_apply(h, 1, qax.QAX_MIXED, v1, o1, 1)
        v8 = torch.randn(N * 8, dtype=torch.complex128, generator=g).to(dev)
        o8 = torch.zeros_like(v8)
        qax.qax_block_apply(h, 1, qax.QAX_FP64, v8, o8, 8)
        qax.qax_block_apply(h, 1, qax.QAX_MIXED, v8, o8, 8)
        torch.cuda.synchronize()
        print("block applies: B, B^-1 FP64, B^-1 FP32; eight columns FP64, FP32", flush=True)
        qax.qax_pair_sum(h, qax.QAX_MIXED, v8, o8, 8)
        torch.cuda.synchronize()
        print("pair sum: FP32, eight right-hand sides", flush=True)
        n = 200
        th = np.linspace(0, 2 * math.pi, n, endpoint=False)
        ph = (np.arange(n) + 0.5) * math.pi / n
        T, P = np.meshgrid(th, ph, indexing="ij")
        xhat = np.stack([np.cos(T) * np.sin(P), np.sin(T) * np.sin(P), np.cos(P)], -1).reshape(-1, 3)
        u = torch.zeros(xhat.shape[0], dtype=torch.complex128, device=dev)
        qax.qax_farfield(h, v1, xhat, u)
        torch.cuda.synchronize()
        print("far field: 40000 directions", flush=True)
    finally:
        qax.qax_destroy(h)
    print("done", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1] if len(sys.argv) > 1 and sys.argv[1] != "-" else None,
                  sys.argv[2] if len(sys.argv) > 2 else "random_mixed"))
