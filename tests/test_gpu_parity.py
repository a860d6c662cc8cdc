"""Parity of the HIP path (called through the C interface) with the FP64 CPU
oracle, on the same seeded inputs.

Tolerances (written here, from the precision contract of the solver):
FP64 operator pieces 1e-11 relative (pair sums 1e-12, self-block entries
1e-12 of the block's largest entry), FP64 solutions 1e-11 relative (the
condition number of the second-kind system is O(1)-O(10), solved to a
residual of 1e-12); mixed-precision operator apply 1e-5 and mixed-precision
solution 1e-6, each both in the 2-norm and element by element (largest
difference over the largest reference entry).
"""
import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import modal as omodal
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


def small27(n_panels=1, n_theta=16, k=5.0):
    s = sc.lattice27(n_panels=n_panels, n_theta=n_theta, k=k)
    return s


def lattice8(n_panels=1, n_theta=12, k=3.0):
    """8 bent spheroids on a 2x2x2 lattice of spacing 3 with two distinct
    curvatures and random rotations (congruent bodies share a self block)."""
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
                i += 1
    return sc.Scenario("lattice8", b, np.array([k]), sc.paper_direction(), tol=1e-10)


def oracle_blocks(d, k_per_problem):
    """Oracle self blocks, computed once per distinct body."""
    cache, out = {}, {}
    for bi, body in enumerate(d.bodies):
        p = d.problem[d.offsets[bi]]
        key = (body.shape, body.a, body.c, body.kappa, body.n_panels, body.n_theta, float(k_per_problem[p]))
        if key not in cache:
            cache[key] = oself.self_block(body, float(k_per_problem[p]))
        out[bi] = cache[key]
    return out


# ---------------------------------------------------------------- geometry
@pytest.mark.parametrize("scen", ["tiny", "small27", "mixed"])
def test_nodes_match_oracle(scen):
    s = {"tiny": lambda: sc.tiny(n_bodies=3, n_theta=8, shapes=(0, 1, 2)),
         "small27": small27,
         "mixed": lambda: sc.random_mixed(n_bodies=20, side=14.0)}[scen]()
    d = geo.discretize(s)
    with qax.Problem(s) as P:
        assert P.N == d.pos.shape[0]
        assert np.array_equal(P.offsets, d.offsets)
        pos = torch.zeros(P.N * 3, dtype=torch.float64, device=DEV)
        aw = torch.zeros(P.N * 3, dtype=torch.float64, device=DEV)
        qax.qax_nodes(P.h, pos, aw)
        assert np.abs(t2n(pos).reshape(-1, 3) - d.pos).max() < 1e-13
        assert np.abs(t2n(aw).reshape(-1, 3) - d.aw).max() < 1e-14


# ---------------------------------------------------------------- pair sum
def _mu(n, nrhs=1, seed=0):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs)))


@pytest.mark.parametrize("scen", ["tiny", "small27", "mixed"])
def test_pair_sum_parity_full(scen):
    s = {"tiny": lambda: sc.tiny(n_bodies=3, n_theta=8, shapes=(0, 1, 2), k=3.0),
         "small27": small27,
         "mixed": lambda: sc.random_mixed(n_bodies=24, side=14.0, k=4.0)}[scen]()
    d = geo.discretize(s)
    mu = _mu(d.pos.shape[0])[:, 0]
    ref = opair.pair_sum(d, s.k, mu)
    with qax.Problem(s) as P:
        out = P.vec()
        qax.qax_pair_sum(P.h, qax.QAX_FP64, n2t(mu), out)
        assert rel(t2n(out), ref) < 1e-12
        assert np.abs(t2n(out) - ref).max() < 1e-12 * np.abs(ref).max()
        qax.qax_pair_sum(P.h, qax.QAX_MIXED, n2t(mu), out)
        assert rel(t2n(out), ref) < 1e-5
        assert np.abs(t2n(out) - ref).max() < 1e-5 * np.abs(ref).max()


def test_pair_sum_lattice27_full_size_sampled():
    # the 27-body lattice at its full discretisation (2048 nodes per body),
    # in the launch configuration the benchmark times; sampled target rows
    s = sc.lattice27()
    d = geo.discretize(s)
    mu = _mu(d.pos.shape[0], seed=5)[:, 0]
    rng = np.random.default_rng(1)
    tg = np.sort(rng.choice(d.pos.shape[0], 384, replace=False))
    tg[0], tg[-1] = 0, d.pos.shape[0] - 1
    ref = opair.pair_sum(d, s.k, mu, targets=tg)
    with qax.Problem(s) as P:
        out = P.vec()
        qax.qax_pair_sum(P.h, qax.QAX_FP64, n2t(mu), out)
        o64 = t2n(out)[tg]
        assert rel(o64, ref) < 1e-12
        qax.qax_pair_sum(P.h, qax.QAX_MIXED, n2t(mu), out)
        assert rel(t2n(out)[tg], ref) < 1e-5
        assert np.abs(t2n(out)[tg] - ref).max() < 1e-5 * np.abs(ref).max()


def test_pair_sum_fp32_reciprocal_ragged_blocks():
    # the FP32 one-right-hand-side pair sum evaluates each unordered pair once
    # for both directions, on blocks of 256 nodes: bodies of 96 to 480 nodes
    # (partial blocks and partial 64-source chunks), two problems with
    # different k and a third problem with a single body (no pairs)
    s = sc.tiny(n_bodies=6, n_theta=6, shapes=(0, 1, 2), k=3.0)
    s.bodies["n_panels"] = [1, 5, 3, 2, 4, 1]
    s.bodies["problem"] = [0, 0, 0, 1, 1, 2]
    s.k = np.array([3.0, 6.5, 2.0])
    d = geo.discretize(s)
    mu = _mu(d.pos.shape[0], seed=9)[:, 0]
    ref = opair.pair_sum(d, s.k, mu)
    assert np.all(ref[d.problem == 2] == 0)
    with qax.Problem(s) as P:
        out = P.vec()
        qax.qax_pair_sum(P.h, qax.QAX_MIXED, n2t(mu), out)
        got = t2n(out)
        assert rel(got, ref) < 1e-5
        assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()
        assert np.all(got[d.problem == 2] == 0)
        for p in (0, 1):
            sel = d.problem == p
            assert rel(got[sel], ref[sel]) < 1e-5
            assert np.abs(got[sel] - ref[sel]).max() < 1e-5 * np.abs(ref[sel]).max()
        # a fixed summation order: a second call gives the same bits
        qax.qax_pair_sum(P.h, qax.QAX_MIXED, n2t(mu), out)
        assert np.array_equal(t2n(out), got)


def test_pair_sum_multi_rhs_and_problems():
    s = sc.tiny(n_bodies=4, n_theta=8, k=2.0)
    s.bodies["problem"] = [0, 0, 1, 1]
    s.k = np.array([2.0, 7.0])
    d = geo.discretize(s)
    nrhs = 5
    mu = _mu(d.pos.shape[0], nrhs, seed=2)
    ref = opair.pair_sum(d, s.k, mu)
    with qax.Problem(s) as P:
        out = P.vec(nrhs)
        qax.qax_pair_sum(P.h, qax.QAX_FP64, n2t(mu.ravel()), out, nrhs)
        assert rel(t2n(out).reshape(-1, nrhs), ref) < 1e-12
        qax.qax_pair_sum(P.h, qax.QAX_MIXED, n2t(mu.ravel()), out, nrhs)
        assert rel(t2n(out).reshape(-1, nrhs), ref) < 1e-5
        assert np.abs(t2n(out).reshape(-1, nrhs) - ref).max() < 1e-5 * np.abs(ref).max()


# ---------------------------------------------------------------- modal engine
@pytest.mark.parametrize("k", [0.0, 3.0, 10.0])
def test_modal_modes_gpu_vs_oracle(k):
    rng = np.random.default_rng(7)
    n = 40
    r = rng.uniform(0.05, 0.7, n)
    chim1 = 10.0 ** rng.uniform(-14, math.log10(0.02), n)
    # choose rt and c consistent with chi - 1
    frac = rng.uniform(0, 1, n)
    tot = chim1 * 2 * r * r   # ((r-rt)^2 + c^2) with rt ~ r
    c = np.sqrt(frac * tot)
    rmrt = np.sqrt((1 - frac) * tot) * np.where(rng.uniform(0, 1, n) < 0.5, -1, 1)
    rt = r - rmrt
    chim1 = (rmrt ** 2 + c ** 2) / (2 * r * rt)
    nmax = 17
    A_ref, B_ref = omodal.derivative_modes(k, r, rt, c, 1 + chim1, chim1, nmax, rmrt=rmrt)
    with qax.Problem(sc.tiny(n_bodies=2)) as P:
        A = torch.zeros(n * (nmax + 1), dtype=torch.complex128, device=DEV)
        B = torch.zeros_like(A)
        qax.qax_modal_modes(P.h, n2t(r), n2t(rt), n2t(c), n2t(chim1), n2t(rmrt), k, nmax, A, B)
        A, B = t2n(A).reshape(n, -1), t2n(B).reshape(n, -1)
    for i in range(n):
        sa = np.abs(A_ref[i]).max()
        sb = np.abs(B_ref[i]).max()
        assert np.abs(A[i] - A_ref[i]).max() < 1e-11 * sa, i
        assert np.abs(B[i] - B_ref[i]).max() < 1e-11 * max(sb, 1e-300) + 1e-300, i


# ---------------------------------------------------------------- self blocks
SELF_CASES = [
    ("sphere", geo.SPHERE, 0.5, 0.5, 0.0, 1, 16, 2.0),
    ("spheroid_k0", geo.SPHEROID, 0.5, 1.0, 0.25, 2, 16, 0.0),
    ("peanut_k5", geo.PEANUT, 0.5, 0.3, 0.15, 2, 32, 5.0),
    ("spheroid_3pan", geo.SPHEROID, 0.5, 1.0, 0.3, 3, 12, 4.0),
]


@pytest.mark.parametrize("case", SELF_CASES, ids=[c[0] for c in SELF_CASES])
def test_self_block_parity(case):
    _, shape, a, c, kap, npan, nth, k = case
    s = sc.tiny(n_bodies=1, n_panels=npan, n_theta=nth, k=k, shapes=(shape,))
    s.bodies["a"], s.bodies["c"], s.bodies["kappa"] = a, c, kap
    disc = geo.discretize_body(shape, a, c, kap, npan, nth)
    n = disc.n
    rows = np.unique(np.concatenate([np.arange(0, n, max(1, n // 12)), [n - 1, nth // 2]]))
    ref = oself.self_block(disc, k, rows=rows)
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        Bt = torch.zeros(n * n, dtype=torch.complex128, device=DEV)
        qax.qax_self_block(P.h, 0, Bt)
        Bg = t2n(Bt).reshape(n, n)
        Bi = torch.zeros_like(Bt)
        qax.qax_self_block(P.h, 0, Bi, inverse=True)
        Binv = t2n(Bi).reshape(n, n)
    err = np.abs(Bg[rows] - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err
    if k > 0:   # at k = 0 the block is singular: (1/2 + D_0)[1] = 0
        assert np.abs(Binv @ Bg - np.eye(n)).max() < 1e-11


def test_self_block_gauss_identity_gpu():
    # (1/2 + D_0)[1] = 0 on a bent peanut, k = 0, directly on the GPU block
    s = sc.tiny(n_bodies=1, n_panels=2, n_theta=20, k=0.0, shapes=(geo.PEANUT,))
    s.bodies["kappa"] = 0.3
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        n = P.N
        Bt = torch.zeros(n * n, dtype=torch.complex128, device=DEV)
        qax.qax_self_block(P.h, 0, Bt)
        Bg = t2n(Bt).reshape(n, n)
    assert np.abs(Bg @ np.ones(n)).max() < 1e-12


# ---------------------------------------------------------------- apply / solve
@pytest.fixture(scope="module")
def small27_oracle():
    s = lattice8()
    d = geo.discretize(s)
    blocks = oracle_blocks(d, s.k)
    return s, d, blocks


def test_apply_parity(small27_oracle):
    s, d, blocks = small27_oracle
    mu = _mu(d.pos.shape[0], seed=11)[:, 0]
    ref = osolve.apply_operator(d, s.k, blocks, mu)
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        out = P.vec()
        qax.qax_apply(P.h, qax.QAX_FP64, n2t(mu), out)
        assert rel(t2n(out), ref) < 1e-11
        qax.qax_apply(P.h, qax.QAX_MIXED, n2t(mu), out)
        assert rel(t2n(out), ref) < 1e-5
        assert np.abs(t2n(out) - ref).max() < 1e-5 * np.abs(ref).max()
        # block-inverse apply undoes the block apply
        v = P.vec()
        qax.qax_block_apply(P.h, 0, qax.QAX_FP64, n2t(mu), v)
        w = P.vec()
        qax.qax_block_apply(P.h, 1, qax.QAX_FP64, v, w)
        assert rel(t2n(w), mu) < 1e-12
        qax.qax_block_apply(P.h, 1, qax.QAX_MIXED, v, w)
        assert rel(t2n(w), mu) < 1e-5
        assert np.abs(t2n(w) - mu).max() < 1e-5 * np.abs(mu).max()


def test_rhs_and_farfield_parity(small27_oracle):
    s, d, blocks = small27_oracle
    b_ref = osolve.rhs_planewave(d, s.k, s.dirs)[:, 0]
    mu = _mu(d.pos.shape[0], seed=4)[:, 0]
    xh = np.array([[0, 0, 1.0], [0.6, 0.8, 0.0], [-0.48, 0.6, 0.64]])
    u_ref = osolve.far_field(d, s.k, mu, xh)
    with qax.Problem(s) as P:
        b = P.vec()
        dirs, nrhs = P.dirs()
        qax.qax_rhs(P.h, dirs, b, nrhs)
        assert np.abs(t2n(b) - b_ref).max() < 1e-13
        u = torch.zeros(3, dtype=torch.complex128, device=DEV)
        qax.qax_farfield(P.h, n2t(mu), xh, u)
        assert rel(t2n(u), u_ref) < 1e-12


@pytest.mark.parametrize("form", ["double", "combined"])
def test_farfield_every_problem(form):
    # three independent problems with their own k: the far field of each
    # problem's density, against the oracle element by element
    s = sc.tiny(n_bodies=6, n_theta=8, shapes=(0, 1, 2), k=3.0)
    s.bodies["problem"] = [0, 0, 1, 1, 1, 2]
    s.k = np.array([3.0, 6.5, 2.0])
    d = geo.discretize(s)
    mu = _mu(d.pos.shape[0], 2, seed=12)
    rng = np.random.default_rng(5)
    xh = rng.standard_normal((7, 3))
    xh /= np.linalg.norm(xh, axis=1)[:, None]
    kw = {"double": {}, "combined": {"formulation": qax.QAX_COMBINED_FIELD, "eta": 1.5}}[form]
    with qax.Problem(s, **kw) as P:
        u = torch.zeros(3 * 7 * 2, dtype=torch.complex128, device=DEV)
        qax.qax_farfield(P.h, n2t(mu.ravel()), xh, u, nrhs=2)
        got = t2n(u).reshape(3, 7, 2)
    for p in range(3):
        for r in range(2):
            want = osolve.far_field(d, s.k, mu[:, r], xh, eta=1.5 if form == "combined" else None, problem=p)
            assert np.abs(got[p, :, r] - want).max() < 1e-12 * np.abs(want).max(), (p, r)


@pytest.mark.parametrize("form", ["double", "combined", "single"])
def test_farfield_antipodal_pairs(small27_oracle, form):
    # directions whose exact negation is also in the list share one phase
    # evaluation: against the oracle, and bitwise equal to one call per
    # direction (the reduction of the half-revolution phase is odd/even)
    s, d, _ = small27_oracle
    mu = _mu(d.pos.shape[0], seed=6)[:, 0]
    rng = np.random.default_rng(3)
    v = rng.standard_normal((5, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    xh = np.concatenate([v, -v[[2, 0, 4]], [[0.0, 0.0, 1.0]], -v[[1]]])   # 4 pairs, 1 alone
    kw = {"double": {}, "combined": {"formulation": qax.QAX_COMBINED_FIELD},
          "single": {"formulation": qax.QAX_SINGLE_LAYER}}[form]
    eta = {"double": None, "combined": s.k[0], "single": None}[form]
    u_ref = osolve.far_field(d, s.k, mu, xh, eta=eta, single=form == "single")
    with qax.Problem(s, **kw) as P:
        u = torch.zeros(xh.shape[0], dtype=torch.complex128, device=DEV)
        qax.qax_farfield(P.h, n2t(mu), xh, u)
        got = t2n(u)
        assert rel(got, u_ref) < 1e-12
        for i in range(xh.shape[0]):
            one = torch.zeros(1, dtype=torch.complex128, device=DEV)
            qax.qax_farfield(P.h, n2t(mu), np.ascontiguousarray(xh[i:i + 1]), one)
            assert t2n(one)[0] == got[i]


def test_solve_parity_fp64_and_mixed(small27_oracle):
    s, d, blocks = small27_oracle
    b = osolve.rhs_planewave(d, s.k, s.dirs)[:, 0]
    x_ref, _, _ = osolve.solve(d, s.k, blocks, b, method="dense")
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        dirs, nrhs = P.dirs()
        x = P.vec()
        info = qax.qax_solve(P.h, qax.QAX_FP64, dirs, x, nrhs, tol=1e-12, maxit=300)
        assert info["rel_res"] <= 1e-12
        assert rel(t2n(x), x_ref) < 1e-11, rel(t2n(x), x_ref)
        assert np.abs(t2n(x) - x_ref).max() < 1e-11 * np.abs(x_ref).max()
        info = qax.qax_solve(P.h, qax.QAX_MIXED, dirs, x, nrhs, tol=1e-8, maxit=300)
        assert info["rel_res"] <= 1e-8
        assert rel(t2n(x), x_ref) < 1e-6
        assert np.abs(t2n(x) - x_ref).max() < 1e-6 * np.abs(x_ref).max()
        assert info["outer_iters"] >= 1


def test_dense_two_spheres_and_mie():
    # the two-sphere workload: 16 GL x 32 azimuths per sphere, k = 2, dense solve
    s = sc.two_spheres()
    d = geo.discretize(s)
    blocks = oracle_blocks(d, s.k)
    b = osolve.rhs_planewave(d, s.k, s.dirs)[:, 0]
    x_ref, _, _ = osolve.solve(d, s.k, blocks, b, method="dense")
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        dirs, nrhs = P.dirs()
        x = P.vec()
        qax.qax_solve_dense(P.h, dirs, x, nrhs)
        assert rel(t2n(x), x_ref) < 1e-11, rel(t2n(x), x_ref)
        assert np.abs(t2n(x) - x_ref).max() < 1e-11 * np.abs(x_ref).max()
        x2 = P.vec()
        qax.qax_solve(P.h, qax.QAX_FP64, dirs, x2, nrhs, tol=1e-12)
        assert rel(t2n(x2), x_ref) < 1e-11, rel(t2n(x2), x_ref)
    # single sphere against the Mie series
    s1 = sc.single_sphere(0.5, 2, 16, 2.0)
    g = np.array([0.0, math.pi / 2, math.pi])
    xh = np.stack([np.sin(g), 0 * g, np.cos(g)], axis=1)
    from scipy.special import eval_legendre, spherical_jn, spherical_yn
    mie = np.zeros(3, dtype=complex)
    for n in range(40):
        hn = spherical_jn(n, 1.0) + 1j * spherical_yn(n, 1.0)
        mie += (2 * n + 1) * spherical_jn(n, 1.0) / hn * eval_legendre(n, np.cos(g))
    mie *= 1j / 2.0
    with qax.Problem(s1) as P:
        qax.qax_assemble_self(P.h)
        dirs, nrhs = P.dirs()
        x = P.vec()
        qax.qax_solve_dense(P.h, dirs, x, nrhs)
        u = torch.zeros(3, dtype=torch.complex128, device=DEV)
        qax.qax_farfield(P.h, x, xh, u)
        assert np.abs(t2n(u) - mie).max() < 1e-10


# ---------------------------------------------------------------- errors
def test_error_paths():
    s = sc.tiny(n_bodies=2)
    P = qax.Problem(s)
    try:
        out = P.vec()
        with pytest.raises(qax.QaxError) as e:
            qax.qax_apply(P.h, qax.QAX_FP64, out, out)
        assert e.value.status == qax.QAX_ERR_STATE
        with pytest.raises(qax.QaxError) as e:
            qax.qax_pair_sum(P.h, qax.QAX_FP64, out, out, nrhs=0)
        assert e.value.status == qax.QAX_ERR_ARG
        bad = s.bodies.copy()
        bad["n_theta"] = 7
        with pytest.raises(qax.QaxError) as e:
            qax.qax_build(P.h, bad, s.k)
        assert e.value.status == qax.QAX_ERR_ARG
        bad = s.bodies.copy()
        bad["cx"][0] = float("nan")
        with pytest.raises(qax.QaxError) as e:
            qax.qax_build(P.h, bad, s.k)
        assert e.value.status == qax.QAX_ERR_ARG
    finally:
        P.close()
