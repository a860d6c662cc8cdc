"""Turn rocprofv3 CSV output of the profiling workload into the per-kernel
summary used by bench.py (HBM traffic per launch) and the markdown table.

    python -m paper_2606_31380_amd.profile_summary <dir> <out.json> <out.md>

<dir> holds the sub-directories trace/ (--kernel-trace --stats), fetch/
(--pmc FETCH_SIZE), write/ (--pmc WRITE_SIZE), valu32/ (F32 VALU instruction
counters), valu64/ (F64 VALU and MFMA counters) and, when present, mfma32/
(SQ_INSTS_VALU_MFMA_MOPS_F32), each with run_*.csv (trace/ also with
run_kernel_trace.csv).  The
memory counters are scaled by what they read for the calibration kernel
(y = 2 x over 2^27 doubles: 1 GiB read and 1 GiB written).  FLOP counts take
64 lanes per VALU instruction and two flops per FMA; MFMA MOPS count 512
flops each.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CAL_BYTES = 1 << 30

# timing kind -> (kernel name pattern as rocprofv3 prints it, source file,
# largest grids only); the single-right-hand-side instance with the most
# launches is taken (the FP32 preconditioner apply: the reduced-inverse
# product when every block is mirror-symmetric).  The inversion's update kernel also runs the 64-column
# sibling updates inside the panel factorization: the trailing updates are its
# dispatches with the largest grid.
KINDS = {
    "pair_sum_fp32": (r"qax::pair_sum_f32_sym_kernel<0>", "paper_2606_31380_amd/csrc/pairsum.hip", False),
    "pair_sum_fp64": (r"qax::pair_sum_f64_sym_kernel<0>", "paper_2606_31380_amd/csrc/pairsum.hip", False),
    "block_apply": (r"qax::block_gemv_kernel<double, 1, \d, \d+>", "paper_2606_31380_amd/csrc/dense.hip", False),
    "block_apply_f32": (r"qax::(block_gemv_f32_lds_kernel<\d>|sym_seg_gemv_kernel<float, 4>)",
                        "paper_2606_31380_amd/csrc/dense.hip", False),
    "self_assembly": (r"qax::assemble_self_kernel<0>", "paper_2606_31380_amd/csrc/selfblock.hip", False),
    "invert_update": (r"qax::gjm_update_kernel<double>", "paper_2606_31380_amd/csrc/dense.hip", True),
}


def short(name: str) -> str:
    name = re.sub(r"\(.*", "", name)
    return name.replace("void ", "").strip()


def load_counters(path, largest=False):
    """Per kernel name: counter values averaged over its dispatches (with
    largest, over the dispatches of its largest grid only)."""
    rows = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            rows[short(r["Kernel_Name"])].append(r)
    out = {}
    for k, rs in rows.items():
        if largest:
            g = max(int(r["Grid_Size"]) for r in rs)
            rs = [r for r in rs if int(r["Grid_Size"]) == g]
        agg = collections.defaultdict(float)
        for r in rs:
            agg[r["Counter_Name"]] += float(r["Counter_Value"])
        n = len({r["Dispatch_Id"] for r in rs})
        out[k] = {c: v / n for c, v in agg.items()}
    return out


def trace_largest(path):
    """Per kernel name: (calls, average us) over the dispatches of its largest grid."""
    d = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            d[short(r["Kernel_Name"])].append((g, int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = {}
    for k, v in d.items():
        g = max(x[0] for x in v)
        ts = [x[1] for x in v if x[0] == g]
        out[k] = (len(ts), sum(ts) / len(ts) / 1e3)
    return out


def sha256(rel):
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def main(d, out_json, out_md):
    trace = {}
    with open(os.path.join(d, "trace", "run_kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            trace[short(r["Name"])] = (int(r["Calls"]), float(r["AverageNs"]) / 1e3)
    passes = {"fetch": "fetch", "write": "write", "v32": "valu32", "v64": "valu64", "m32": "mfma32"}
    cnt = {}
    for largest in (False, True):
        for key, sub in passes.items():
            path = os.path.join(d, sub, "run_counter_collection.csv")
            cnt[key, largest] = load_counters(path, largest) if os.path.exists(path) else {}
    fetch, write = cnt["fetch", False], cnt["write", False]
    tlarge = trace_largest(os.path.join(d, "trace", "run_kernel_trace.csv"))
    cal = next(k for k in fetch if "MulFunctor" in k)
    f_fetch = CAL_BYTES / (fetch[cal]["FETCH_SIZE"] * 1024)
    f_write = CAL_BYTES / (write[cal]["WRITE_SIZE"] * 1024)

    def row(k, largest=False):
        fetch, write = cnt["fetch", largest], cnt["write", largest]
        v32, v64, m32 = cnt["v32", largest], cnt["v64", largest], cnt["m32", largest]
        tr = tlarge if largest else trace
        g = v32.get(k, {})
        h = v64.get(k, {})
        f32 = 64 * (g.get("SQ_INSTS_VALU_ADD_F32", 0) + g.get("SQ_INSTS_VALU_MUL_F32", 0)
                    + g.get("SQ_INSTS_VALU_TRANS_F32", 0) + 2 * g.get("SQ_INSTS_VALU_FMA_F32", 0))
        f64 = 64 * (h.get("SQ_INSTS_VALU_ADD_F64", 0) + h.get("SQ_INSTS_VALU_MUL_F64", 0)
                    + h.get("SQ_INSTS_VALU_TRANS_F64", 0) + 2 * h.get("SQ_INSTS_VALU_FMA_F64", 0))
        return {
            "calls": tr.get(k, (0, 0.0))[0], "avg_us": tr.get(k, (0, 0.0))[1],
            "fetch_bytes": fetch.get(k, {}).get("FETCH_SIZE", 0.0) * 1024 * f_fetch,
            "write_bytes": write.get(k, {}).get("WRITE_SIZE", 0.0) * 1024 * f_write,
            "valu_insts": g.get("SQ_INSTS_VALU", 0.0), "valu_trans_f32": g.get("SQ_INSTS_VALU_TRANS_F32", 0.0),
            "f32_flop": f32, "f64_flop": f64,
            "mfma_f64_flop": 512 * h.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0),
            "mfma_f32_flop": 512 * m32.get(k, {}).get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0),
        }

    out = {"calibration": {"kernel": cal, "bytes_read": CAL_BYTES, "bytes_written": CAL_BYTES,
                           "fetch_size_kib": fetch[cal]["FETCH_SIZE"], "write_size_kib": write[cal]["WRITE_SIZE"],
                           "fetch_factor": f_fetch, "write_factor": f_write},
           "kernels": {}}
    for kind, (pattern, src, largest) in KINDS.items():
        names = [k for k in fetch if re.fullmatch(pattern, k)]
        if names:
            kname = max(names, key=lambda k: trace.get(k, (0, 0.0))[0])
            out["kernels"][kind] = dict(row(kname, largest), kernel=kname, source=src,
                                        source_sha256=sha256(src), largest_grid_only=largest)
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    lines = ["| kernel | calls | avg us | HBM read MB | HBM write MB | VALU insts | F32 flop | F64 flop | MFMA F64 flop | MFMA F32 flop |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(trace, key=lambda k: -trace[k][0] * trace[k][1]):
        if k not in fetch:
            continue
        r = row(k)
        lines.append(f"| `{k[:70]}` | {r['calls']} | {r['avg_us']:.1f} | {r['fetch_bytes'] / 1e6:.2f} | "
                     f"{r['write_bytes'] / 1e6:.2f} | {r['valu_insts']:.3e} | {r['f32_flop']:.3e} | "
                     f"{r['f64_flop']:.3e} | {r['mfma_f64_flop']:.3e} | {r['mfma_f32_flop']:.3e} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"calibration factors: FETCH_SIZE x{f_fetch:.4f}, WRITE_SIZE x{f_write:.4f}")


if __name__ == "__main__":
    main(*sys.argv[1:4])
