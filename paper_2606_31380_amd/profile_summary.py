"""Turn rocprofv3 CSV output of the profiling workload into the per-kernel
summary used by bench.py (HBM traffic per launch) and the markdown table.

    python -m paper_2606_31380_amd.profile_summary <dir> <out.json> <out.md>

<dir> holds the sub-directories trace/ (--kernel-trace --stats), fetch/
(--pmc FETCH_SIZE), write/ (--pmc WRITE_SIZE), valu32/ (F32 VALU instruction
counters), valu64/ (F64 VALU and MFMA counters) and, when present, mfma32/
(SQ_INSTS_VALU_MFMA_MOPS_F32), each with run_*.csv.  The
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

# timing kind -> (kernel name pattern as rocprofv3 prints it, source file); the
# single-right-hand-side instance with the most launches is taken
KINDS = {
    "pair_sum_fp32": (r"qax::pair_sum_f32_kernel<\d+, 1, 0>", "paper_2606_31380_amd/csrc/pairsum.hip"),
    "pair_sum_fp64": (r"qax::pair_sum_f64_kernel<\d+, 1, 0>", "paper_2606_31380_amd/csrc/pairsum.hip"),
    "block_apply": (r"qax::block_gemv_kernel<double, 1, \d, \d+>", "paper_2606_31380_amd/csrc/dense.hip"),
    "block_apply_f32": (r"qax::block_gemv_f32_lds_kernel<\d>", "paper_2606_31380_amd/csrc/dense.hip"),
    "self_assembly": (r"qax::assemble_self_kernel<0>", "paper_2606_31380_amd/csrc/selfblock.hip"),
    "invert_update": (r"qax::gjm_update_kernel<float>", "paper_2606_31380_amd/csrc/dense.hip"),
}


def short(name: str) -> str:
    name = re.sub(r"\(.*", "", name)
    return name.replace("void ", "").strip()


def load_counters(path):
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    with open(path) as f:
        for r in csv.DictReader(f):
            k = short(r["Kernel_Name"])
            agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[k].add(r["Dispatch_Id"])
    return {k: {c: v / len(disp[k]) for c, v in d.items()} for k, d in agg.items()}


def sha256(rel):
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def main(d, out_json, out_md):
    trace = {}
    with open(os.path.join(d, "trace", "run_kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            trace[short(r["Name"])] = (int(r["Calls"]), float(r["AverageNs"]) / 1e3)
    fetch = load_counters(os.path.join(d, "fetch", "run_counter_collection.csv"))
    write = load_counters(os.path.join(d, "write", "run_counter_collection.csv"))
    v32 = load_counters(os.path.join(d, "valu32", "run_counter_collection.csv"))
    v64 = load_counters(os.path.join(d, "valu64", "run_counter_collection.csv"))
    m32_path = os.path.join(d, "mfma32", "run_counter_collection.csv")
    m32 = load_counters(m32_path) if os.path.exists(m32_path) else {}
    cal = next(k for k in fetch if "MulFunctor" in k)
    f_fetch = CAL_BYTES / (fetch[cal]["FETCH_SIZE"] * 1024)
    f_write = CAL_BYTES / (write[cal]["WRITE_SIZE"] * 1024)

    def row(k):
        g = v32.get(k, {})
        h = v64.get(k, {})
        f32 = 64 * (g.get("SQ_INSTS_VALU_ADD_F32", 0) + g.get("SQ_INSTS_VALU_MUL_F32", 0)
                    + g.get("SQ_INSTS_VALU_TRANS_F32", 0) + 2 * g.get("SQ_INSTS_VALU_FMA_F32", 0))
        f64 = 64 * (h.get("SQ_INSTS_VALU_ADD_F64", 0) + h.get("SQ_INSTS_VALU_MUL_F64", 0)
                    + h.get("SQ_INSTS_VALU_TRANS_F64", 0) + 2 * h.get("SQ_INSTS_VALU_FMA_F64", 0))
        return {
            "calls": trace.get(k, (0, 0.0))[0], "avg_us": trace.get(k, (0, 0.0))[1],
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
    for kind, (pattern, src) in KINDS.items():
        names = [k for k in fetch if re.fullmatch(pattern, k)]
        if names:
            kname = max(names, key=lambda k: trace.get(k, (0, 0.0))[0])
            out["kernels"][kind] = dict(row(kname), kernel=kname, source=src, source_sha256=sha256(src))
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
