"""Thin ctypes binding of libqax (include/qax.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Functions carry the C names; device arrays are torch tensors on the handle's
device (complex128 unless stated), host arrays are numpy arrays.  If the
library is not built, loading fails loudly -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqax.so")

QAX_OK, QAX_ERR_ARG, QAX_ERR_DEVICE, QAX_ERR_NOMEM, QAX_ERR_NOCONV, QAX_ERR_STATE = range(6)
QAX_FP64, QAX_MIXED = 0, 1
QAX_DOUBLE_LAYER, QAX_COMBINED_FIELD, QAX_SINGLE_LAYER = 0, 1, 2
QAX_SOLVER_LOCKSTEP, QAX_SOLVER_BLOCK = 0, 1
STATUS_NAMES = {0: "QAX_OK", 1: "QAX_ERR_ARG", 2: "QAX_ERR_DEVICE", 3: "QAX_ERR_NOMEM",
                4: "QAX_ERR_NOCONV", 5: "QAX_ERR_STATE"}


class qax_body(C.Structure):
    _fields_ = [("shape", C.c_int32), ("n_panels", C.c_int32), ("n_theta", C.c_int32),
                ("problem", C.c_int32), ("a", C.c_double), ("c", C.c_double),
                ("kappa", C.c_double), ("theta1", C.c_double), ("theta2", C.c_double),
                ("centre", C.c_double * 3), ("n_ref", C.c_int32)]


class qax_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("rel_res", C.c_double),
                ("t_setup_s", C.c_double), ("t_solve_s", C.c_double)]


class qax_tuning_info(C.Structure):
    _fields_ = [("tuned", C.c_int32), ("from_cache", C.c_int32), ("pair_tpb", C.c_int32 * 2),
                ("pair_slot_mult", C.c_int32 * 2), ("pair_nrc", (C.c_int32 * 4) * 2),
                ("gemv_vec", C.c_int32 * 2), ("pair_ms", C.c_double * 2),
                ("default_pair_ms", C.c_double * 2), ("pair_sym_s", C.c_int32 * 2)]


class QaxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_LIB = None
EXPORTS = ["qax_create", "qax_destroy", "qax_last_error", "qax_build", "qax_size", "qax_nodes",
           "qax_assemble_self", "qax_self_block", "qax_pair_sum", "qax_block_apply", "qax_apply",
           "qax_rhs", "qax_solve", "qax_solve_dense", "qax_farfield", "qax_modal_modes",
           "qax_set_timing", "qax_timing", "qax_autotune", "qax_tuning", "qax_set_tuning", "qax_set_graphs",
           "qax_solve_rhs", "qax_nearfield", "qax_set_formulation", "qax_lattice", "qax_invert",
           "qax_set_factorization", "qax_farfield_noalloc", "qax_set_solver"]
(QAX_K_PAIRSUM_FP64, QAX_K_PAIRSUM_FP32, QAX_K_BLOCK_APPLY, QAX_K_SELF_ASSEMBLY, QAX_K_INVERT,
 QAX_K_INVERT_UPDATE, QAX_K_BLOCK_APPLY_F32, QAX_K_LATTICE_F64, QAX_K_LATTICE_F32) = range(9)
KERNEL_NAMES = ["pair_sum_fp64", "pair_sum_fp32", "block_apply", "self_assembly", "invert",
                "invert_update", "block_apply_f32", "lattice_f64", "lattice_f32"]


def lib():
    """Load libqax.so (built in-tree by paper_2606_31380_amd.build)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2606_31380_amd.build`")
    # torch first: its HIP runtime (same SONAME as the system one) is then the
    # single runtime of the process, shared with the library's kernels.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pd = C.POINTER(C.c_double)
    sig = {
        "qax_create": (C.c_int, [C.c_int, vp, C.POINTER(vp)]),
        "qax_destroy": (None, [vp]),
        "qax_last_error": (C.c_char_p, [vp]),
        "qax_build": (C.c_int, [vp, C.POINTER(qax_body), i32, pd, i32]),
        "qax_size": (C.c_int, [vp, C.POINTER(i64), C.POINTER(i64)]),
        "qax_nodes": (C.c_int, [vp, vp, vp]),
        "qax_assemble_self": (C.c_int, [vp, pd]),
        "qax_self_block": (C.c_int, [vp, i32, i32, vp]),
        "qax_pair_sum": (C.c_int, [vp, C.c_int, vp, vp, i32]),
        "qax_block_apply": (C.c_int, [vp, i32, C.c_int, vp, vp, i32]),
        "qax_apply": (C.c_int, [vp, C.c_int, vp, vp, i32]),
        "qax_rhs": (C.c_int, [vp, pd, i32, vp]),
        "qax_solve": (C.c_int, [vp, C.c_int, pd, i32, d, i32, vp, C.POINTER(qax_info)]),
        "qax_solve_dense": (C.c_int, [vp, pd, i32, vp]),
        "qax_invert": (C.c_int, [vp, C.c_int, i32, C.POINTER(i32), vp]),
        "qax_solve_rhs": (C.c_int, [vp, C.c_int, vp, i32, d, i32, vp, C.POINTER(qax_info)]),
        "qax_nearfield": (C.c_int, [vp, vp, i32, pd, i64, i32, vp]),
        "qax_farfield": (C.c_int, [vp, vp, i32, pd, i32, vp]),
        "qax_farfield_noalloc": (C.c_int, [vp, vp, i32, vp, i32, vp]),
        "qax_modal_modes": (C.c_int, [vp, i32, vp, vp, vp, vp, vp, d, i32, vp, vp]),
        "qax_set_timing": (C.c_int, [vp, i32]),
        "qax_set_graphs": (C.c_int, [vp, i32]),
        "qax_set_formulation": (C.c_int, [vp, i32, C.c_double]),
        "qax_set_factorization": (C.c_int, [vp, C.c_int]),
        "qax_set_solver": (C.c_int, [vp, i32]),
        "qax_lattice": (C.c_int, [vp, i32, C.POINTER(i32)]),
        "qax_timing": (C.c_int, [vp, i32, C.POINTER(i64), pd]),
        "qax_autotune": (C.c_int, [vp, i32, C.c_char_p]),
        "qax_tuning": (C.c_int, [vp, C.POINTER(qax_tuning_info)]),
        "qax_set_tuning": (C.c_int, [vp, C.POINTER(qax_tuning_info)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(h, st):
    if st != QAX_OK:
        raise QaxError(st, lib().qax_last_error(h).decode())


def bodies_to_c(bodies) -> "C.Array":
    """Marshal BODY_DTYPE records (paper_2606_31380_amd.scenarios) into qax_body[]."""
    arr = (qax_body * len(bodies))()
    for i, b in enumerate(bodies):
        arr[i].shape = int(b["shape"])
        arr[i].n_panels = int(b["n_panels"])
        arr[i].n_theta = int(b["n_theta"])
        arr[i].problem = int(b["problem"])
        arr[i].a, arr[i].c, arr[i].kappa = float(b["a"]), float(b["c"]), float(b["kappa"])
        arr[i].theta1, arr[i].theta2 = float(b["theta1"]), float(b["theta2"])
        arr[i].centre[0], arr[i].centre[1], arr[i].centre[2] = float(b["cx"]), float(b["cy"]), float(b["cz"])
        arr[i].n_ref = int(b["n_ref"]) if "n_ref" in b.dtype.names else 0
    return arr


# ---------------------------------------------------------------- C names
def qax_create(device=0, stream=None):
    h = C.c_void_p()
    st = lib().qax_create(int(device), C.c_void_p(stream) if stream else None, C.byref(h))
    if st != QAX_OK:
        raise QaxError(st, "qax_create failed")
    return h


def qax_destroy(h):
    lib().qax_destroy(h)


def qax_build(h, bodies, k_per_problem):
    cb = bodies_to_c(bodies)
    k = np.ascontiguousarray(k_per_problem, dtype=np.float64)
    _check(h, lib().qax_build(h, cb, len(bodies), _dptr(k), k.shape[0]))


def qax_size(h, n_bodies=None):
    n = C.c_int64()
    off = None
    if n_bodies is not None:
        off = np.zeros(n_bodies + 1, dtype=np.int64)
        _check(h, lib().qax_size(h, C.byref(n), off.ctypes.data_as(C.POINTER(C.c_int64))))
    else:
        _check(h, lib().qax_size(h, C.byref(n), None))
    return n.value, off


def qax_nodes(h, pos, aw):
    _check(h, lib().qax_nodes(h, _ptr(pos), _ptr(aw)))


def qax_assemble_self(h):
    t = C.c_double()
    _check(h, lib().qax_assemble_self(h, C.byref(t)))
    return t.value


def qax_self_block(h, body, out, inverse=False):
    _check(h, lib().qax_self_block(h, int(body), int(bool(inverse)), _ptr(out)))


def qax_pair_sum(h, prec, mu, out, nrhs=1):
    _check(h, lib().qax_pair_sum(h, int(prec), _ptr(mu), _ptr(out), int(nrhs)))


def qax_block_apply(h, inverse, prec, v, out, nrhs=1):
    _check(h, lib().qax_block_apply(h, int(bool(inverse)), int(prec), _ptr(v), _ptr(out), int(nrhs)))


def qax_apply(h, prec, mu, out, nrhs=1):
    _check(h, lib().qax_apply(h, int(prec), _ptr(mu), _ptr(out), int(nrhs)))


def qax_rhs(h, dirs, out, nrhs=1):
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    _check(h, lib().qax_rhs(h, _dptr(d), int(nrhs), _ptr(out)))


def qax_solve(h, prec, dirs, mu_out, nrhs=1, tol=1e-8, maxit=500, raise_noconv=True):
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    info = qax_info()
    st = lib().qax_solve(h, int(prec), _dptr(d), int(nrhs), float(tol), int(maxit), _ptr(mu_out),
                         C.byref(info))
    if st != QAX_OK and (st != QAX_ERR_NOCONV or raise_noconv):
        _check(h, st)
    return {"status": st, "iters": info.iters, "outer_iters": info.outer_iters,
            "rel_res": info.rel_res, "t_solve_s": info.t_solve_s}


def qax_solve_rhs(h, prec, rhs, mu_out, nrhs=1, tol=1e-8, maxit=500, raise_noconv=True):
    info = qax_info()
    st = lib().qax_solve_rhs(h, int(prec), _ptr(rhs), int(nrhs), float(tol), int(maxit),
                             _ptr(mu_out), C.byref(info))
    if st != QAX_OK and (st != QAX_ERR_NOCONV or raise_noconv):
        _check(h, st)
    return {"status": st, "iters": info.iters, "outer_iters": info.outer_iters,
            "rel_res": info.rel_res, "t_solve_s": info.t_solve_s}


def qax_nearfield(h, mu, pts, u, nrhs=1, problem=0):
    x = np.ascontiguousarray(pts, dtype=np.float64)
    _check(h, lib().qax_nearfield(h, _ptr(mu), int(nrhs), _dptr(x), x.shape[0], int(problem), _ptr(u)))


def qax_solve_dense(h, dirs, mu_out, nrhs=1):
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    _check(h, lib().qax_solve_dense(h, _dptr(d), int(nrhs), _ptr(mu_out)))


def qax_invert(h, prec, orders, mats):
    """Invert in place the complex128 matrices of the given orders stored one
    after another in the device buffer `mats`."""
    o = np.ascontiguousarray(orders, dtype=np.int32)
    _check(h, lib().qax_invert(h, int(prec), int(o.size), o.ctypes.data_as(C.POINTER(C.c_int32)),
                               _ptr(mats)))


def qax_farfield(h, mu, xhat, u_inf, nrhs=1):
    x = np.ascontiguousarray(xhat, dtype=np.float64)
    _check(h, lib().qax_farfield(h, _ptr(mu), int(nrhs), _dptr(x), x.shape[0], _ptr(u_inf)))


def qax_farfield_noalloc(h, mu, d_xhat, u_inf, nrhs=1):
    """Far field with device directions (n_dirs x 3 float64 tensor) and no
    allocation; enqueued on the handle's stream, not waited for."""
    _check(h, lib().qax_farfield_noalloc(h, _ptr(mu), int(nrhs), _ptr(d_xhat), int(d_xhat.shape[0]),
                                         _ptr(u_inf)))


def qax_modal_modes(h, r, rt, c, chim1, rmrt, k, nmax, A, B):
    _check(h, lib().qax_modal_modes(h, int(r.shape[0]), _ptr(r), _ptr(rt), _ptr(c), _ptr(chim1),
                                    _ptr(rmrt), float(k), int(nmax), _ptr(A), _ptr(B)))


def qax_set_graphs(h, enable=True):
    _check(h, lib().qax_set_graphs(h, int(bool(enable))))


def qax_lattice(h, enable=True):
    """Block-Toeplitz inter-body apply on a regular array of identical bodies;
    returns (P, Q, R) when enabled."""
    dims = (C.c_int32 * 3)()
    _check(h, lib().qax_lattice(h, int(bool(enable)), dims))
    return tuple(int(v) for v in dims) if enable else None


def qax_set_formulation(h, formulation, eta=0.0):
    """QAX_DOUBLE_LAYER, QAX_COMBINED_FIELD (eta > 0 fixed coupling, else k)
    or QAX_SINGLE_LAYER."""
    _check(h, lib().qax_set_formulation(h, int(formulation), float(eta)))


def qax_set_factorization(h, prec):
    """QAX_FP64 (default): FP64 inverse, rounded to FP32 for the mixed path;
    QAX_MIXED: inverse computed in FP32."""
    _check(h, lib().qax_set_factorization(h, int(prec)))


def qax_set_solver(h, solver):
    """QAX_SOLVER_LOCKSTEP (default) or QAX_SOLVER_BLOCK (block GMRES) for
    several right-hand sides."""
    _check(h, lib().qax_set_solver(h, int(solver)))


def qax_set_timing(h, enable=True):
    _check(h, lib().qax_set_timing(h, int(bool(enable))))


def qax_timing(h, kernel):
    n = C.c_int64()
    ms = C.c_double()
    _check(h, lib().qax_timing(h, int(kernel), C.byref(n), C.byref(ms)))
    return n.value, ms.value


def qax_autotune(h, nrhs_max=1, cache_path=None):
    cp = None if cache_path is None else os.fsencode(cache_path)
    _check(h, lib().qax_autotune(h, int(nrhs_max), cp))


def qax_tuning(h):
    t = qax_tuning_info()
    _check(h, lib().qax_tuning(h, C.byref(t)))
    return {"tuned": bool(t.tuned), "from_cache": bool(t.from_cache),
            "pair_tpb": {"fp64": t.pair_tpb[0], "fp32": t.pair_tpb[1]},
            "pair_slot_mult": {"fp64": t.pair_slot_mult[0], "fp32": t.pair_slot_mult[1]},
            "pair_nrc": {"fp64": list(t.pair_nrc[0]), "fp32": list(t.pair_nrc[1])},
            "gemv_vec": {"fp64": t.gemv_vec[0], "fp32": t.gemv_vec[1]},
            "pair_ms": {"fp64": t.pair_ms[0], "fp32": t.pair_ms[1]},
            "default_pair_ms": {"fp64": t.default_pair_ms[0], "fp32": t.default_pair_ms[1]},
            "pair_sym_s": {"fp64": t.pair_sym_s[0], "fp32": t.pair_sym_s[1]}}


def qax_set_tuning(h, pair_tpb=(256, 256), pair_slot_mult=(8, 8),
                   pair_nrc=((4, 8, 8, 8), (4, 8, 16, 16)), gemv_vec=(1, 1), pair_sym_s=(0, 0)):
    """Set the launch choices by hand ([FP64, FP32] pairs, as qax_tuning reports)."""
    t = qax_tuning_info()
    for i in range(2):
        t.pair_tpb[i] = int(pair_tpb[i])
        t.pair_slot_mult[i] = int(pair_slot_mult[i])
        for c in range(4):
            t.pair_nrc[i][c] = int(pair_nrc[i][c])
        t.gemv_vec[i] = int(gemv_vec[i])
        t.pair_sym_s[i] = int(pair_sym_s[i])
    _check(h, lib().qax_set_tuning(h, C.byref(t)))


class Problem:
    """Handle + scenario convenience wrapper (marshalling only)."""

    def __init__(self, scenario, device=0, formulation=None, eta=0.0):
        import torch
        self.torch = torch
        self.scenario = scenario
        self.dev = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.dev).cuda_stream
        self.h = qax_create(device, stream)
        if formulation is not None:
            qax_set_formulation(self.h, formulation, eta)
        qax_build(self.h, scenario.bodies, scenario.k)
        self.N, self.offsets = qax_size(self.h, len(scenario.bodies))

    def close(self):
        if self.h is not None:
            qax_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def vec(self, nrhs=1):
        return self.torch.zeros(self.N * nrhs, dtype=self.torch.complex128, device=self.dev)

    def dirs(self, dirs=None):
        s = self.scenario
        d = np.asarray(s.dirs if dirs is None else dirs, dtype=np.float64)
        if "dirs" in s.notes and dirs is None:
            d = np.asarray(s.notes["dirs"], dtype=np.float64)[:, None, :]   # per problem
            return d.reshape(-1, 3), 1
        nrhs = d.shape[0]
        return np.tile(d[None], (s.n_problems, 1, 1)).reshape(-1, 3), nrhs
