"""Batched paths of the HIP library against the oracle and against their
unbatched forms: several right-hand sides (block applies on the matrix cores,
lockstep GMRES) and several independent problems in one call.

Tolerances: FP64 1e-11 (applies; self-block entries 1e-12 of the largest) and
1e-11 (solutions at a residual of 1e-12), FP32 1e-5 / 1e-6 in the 2-norm and
element by element.
"""
import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import pairsum as opair
from oracle import selfblock as oself
from oracle import solve as osolve
from paper_2606_31380_amd import scenarios as sc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_31380_amd import qax  # noqa: E402

DEV = torch.device("cuda", 0)


def t2n(t):
    return t.detach().cpu().numpy()


def n2t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def lattice8(k=3.0, n_theta=12, n_panels=1, problem=0):
    rng = np.random.default_rng(8)
    b = sc.make_bodies(8)
    i = 0
    for x in (0.0, 3.0):
        for y in (0.0, 3.0):
            for z in (0.0, 3.0):
                b[i]["shape"], b[i]["a"], b[i]["c"] = sc.SPHEROID, 0.5, 1.0
                b[i]["kappa"] = (0.1, 0.25)[i % 2]
                b[i]["n_panels"], b[i]["n_theta"] = n_panels, n_theta
                b[i]["theta1"], b[i]["theta2"] = rng.uniform(0, 2 * math.pi, 2)
                b[i]["cx"], b[i]["cy"], b[i]["cz"] = x, y, z
                b[i]["problem"] = problem
                i += 1
    return b


def oracle_blocks(d, k_per_problem):
    cache, out = {}, {}
    for bi, body in enumerate(d.bodies):
        p = d.problem[d.offsets[bi]]
        key = (body.shape, body.a, body.c, body.kappa, body.n_panels, body.n_theta, float(k_per_problem[p]))
        if key not in cache:
            cache[key] = oself.self_block(body, float(k_per_problem[p]))
        out[bi] = cache[key]
    return out


def dirs_on_sphere(n, seed=3):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    s = np.sqrt(1 - u * u)
    return np.stack([s * np.cos(ph), s * np.sin(ph), u], 1)


@pytest.mark.parametrize("nrhs", [4, 8, 37])
def test_block_apply_several_rhs_mfma(nrhs):
    s = sc.Scenario("l8", lattice8(), np.array([3.0]), sc.paper_direction())
    rng = np.random.default_rng(nrhs)
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        N = P.N
        v = rng.standard_normal((N, nrhs)) + 1j * rng.standard_normal((N, nrhs))
        blocks, inv = [], []
        for b in range(8):
            n = P.offsets[b + 1] - P.offsets[b]
            t = torch.zeros(n * n, dtype=torch.complex128, device=DEV)
            qax.qax_self_block(P.h, b, t)
            blocks.append(t2n(t).reshape(n, n))
            qax.qax_self_block(P.h, b, t, inverse=True)
            inv.append(t2n(t).reshape(n, n))
        ref = np.concatenate([blocks[b] @ v[P.offsets[b]:P.offsets[b + 1]] for b in range(8)])
        refi = np.concatenate([inv[b] @ v[P.offsets[b]:P.offsets[b + 1]] for b in range(8)])
        out = P.vec(nrhs)
        qax.qax_block_apply(P.h, 0, qax.QAX_FP64, n2t(v.ravel()), out, nrhs)
        assert rel(t2n(out).reshape(N, nrhs), ref) < 1e-13
        qax.qax_block_apply(P.h, 1, qax.QAX_FP64, n2t(v.ravel()), out, nrhs)
        assert rel(t2n(out).reshape(N, nrhs), refi) < 1e-13
        qax.qax_block_apply(P.h, 1, qax.QAX_MIXED, n2t(v.ravel()), out, nrhs)
        assert rel(t2n(out).reshape(N, nrhs), refi) < 1e-5
        assert np.abs(t2n(out).reshape(N, nrhs) - refi).max() < 1e-5 * np.abs(refi).max()


@pytest.fixture(scope="module")
def l8_oracle():
    s = sc.Scenario("l8", lattice8(), np.array([3.0]), sc.paper_direction())
    d = geo.discretize(s)
    blocks = oracle_blocks(d, s.k)
    A = osolve.dense_matrix_fast(d, s.k, blocks)
    return s, d, blocks, A


def test_solve_several_rhs_lockstep(l8_oracle):
    s, d, blocks, A = l8_oracle
    nrhs = 8
    dirs = dirs_on_sphere(nrhs)
    B = osolve.rhs_planewave(d, s.k, dirs)
    X = np.linalg.solve(A, B)
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        x = P.vec(nrhs)
        info = qax.qax_solve(P.h, qax.QAX_FP64, dirs, x, nrhs, tol=1e-12, maxit=400)
        assert info["rel_res"] <= 1e-12
        assert rel(t2n(x).reshape(-1, nrhs), X) < 1e-11, rel(t2n(x).reshape(-1, nrhs), X)
        info = qax.qax_solve(P.h, qax.QAX_MIXED, dirs, x, nrhs, tol=1e-8, maxit=400)
        assert rel(t2n(x).reshape(-1, nrhs), X) < 1e-6
        assert np.abs(t2n(x).reshape(-1, nrhs) - X).max() < 1e-6 * np.abs(X).max()
        # each column equals its own single-RHS solve
        for r in (0, 5):
            x1 = P.vec(1)
            qax.qax_solve(P.h, qax.QAX_FP64, dirs[r:r + 1], x1, 1, tol=1e-12, maxit=400)
            assert rel(t2n(x1), X[:, r]) < 1e-11


def test_independent_problems_batched_equals_sequential():
    ks = [2.0, 4.5, 7.0]
    rows = [lattice8(k=ks[p], problem=p) for p in range(3)]
    for p, r in enumerate(rows):
        r["cx"] += 0.3 * p                     # different geometry per problem
        r["kappa"] = r["kappa"] * (1 + 0.1 * p)
        r["n_theta"] = (12, 16, 10)[p]
    bodies = np.concatenate(rows)
    dirs = dirs_on_sphere(3, seed=9)           # one direction per problem
    sb = sc.Scenario("batch", bodies, np.array(ks), dirs[:1], notes={"dirs": dirs})
    with qax.Problem(sb) as P:
        qax.qax_assemble_self(P.h)
        dd, nrhs = P.dirs()
        xb = P.vec()
        info = qax.qax_solve(P.h, qax.QAX_FP64, dd, xb, nrhs, tol=1e-12, maxit=400)
        assert info["rel_res"] <= 1e-12
        xb = t2n(xb)
        off = P.offsets
    for p in range(3):
        s1 = sc.Scenario("one", rows[p].copy(), np.array([ks[p]]), dirs[p:p + 1])
        s1.bodies["problem"] = 0
        with qax.Problem(s1) as P1:
            qax.qax_assemble_self(P1.h)
            d1, n1 = P1.dirs()
            x1 = P1.vec()
            qax.qax_solve(P1.h, qax.QAX_FP64, d1, x1, n1, tol=1e-12, maxit=400)
            seg = xb[off[8 * p]:off[8 * p + 8]]
            assert rel(seg, t2n(x1)) < 1e-11, rel(seg, t2n(x1))
    # and the batched pair sum against the oracle
    d = geo.discretize(sb)
    mu = np.cos(np.arange(d.pos.shape[0]) * 0.1) + 0.3j
    with qax.Problem(sb) as P:
        out = P.vec()
        qax.qax_pair_sum(P.h, qax.QAX_FP64, n2t(mu), out)
        assert rel(t2n(out), opair.pair_sum(d, sb.k, mu)) < 1e-12


def test_uneven_mixed_bodies_apply_sampled():
    # uneven discretisations and three shapes (the 1000-body workload's mix)
    s = sc.random_mixed(n_bodies=30, side=16.0, k=4.0, seed=2)
    d = geo.discretize(s)
    mu = np.exp(0.01j * np.arange(d.pos.shape[0]))
    rng = np.random.default_rng(0)
    tg = np.sort(rng.choice(d.pos.shape[0], 200, replace=False))
    ps = opair.pair_sum(d, s.k, mu, targets=tg)
    with qax.Problem(s) as P:
        out = P.vec()
        qax.qax_pair_sum(P.h, qax.QAX_FP64, n2t(mu), out)
        assert rel(t2n(out)[tg], ps) < 1e-12
        qax.qax_pair_sum(P.h, qax.QAX_MIXED, n2t(mu), out)
        assert rel(t2n(out)[tg], ps) < 1e-5
        assert np.abs(t2n(out)[tg] - ps).max() < 1e-5 * np.abs(ps).max()
        qax.qax_assemble_self(P.h)
        # self-block rows of two bodies of different shapes against the oracle
        for bi in (0, 7):
            body = d.bodies[bi]
            n = body.n
            t = torch.zeros(n * n, dtype=torch.complex128, device=DEV)
            qax.qax_self_block(P.h, bi, t)
            rows = np.array([0, n // 3, n - 1])
            ref = oself.self_block(body, 4.0, rows=rows)
            got = t2n(t).reshape(n, n)[rows]
            assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
