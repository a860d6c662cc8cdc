"""Edge cases of the GPU path through the C interface, against the oracle:

* the largest body (8192 nodes: 8 panels x 64 azimuths, and 4 uniform
  panels with 2 refinements per pole x 64 azimuths): self-block rows, the
  FP64 and FP32 inverses, pair sums;
* the fewest azimuths (n_theta = 4, two modes) and a single panel;
* a single body (no inter-body sum), k = 0 next to k > 0 in one batch;
* the largest number of right-hand sides (256);
* argument errors of qax_build for the shape and refinement limits.
"""
import numpy as np
import pytest

from oracle import geometry as geo
from oracle import pairsum as opair
from oracle import selfblock as oself
from paper_2606_31380_amd import scenarios as sc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_31380_amd import qax  # noqa: E402

DEV = torch.device("cuda", 0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def scenario(specs, k=(3.0,), problems=None):
    b = sc.make_bodies(len(specs))
    for i, (shape, a, c, kap, npan, nref, nth) in enumerate(specs):
        b[i]["shape"], b[i]["a"], b[i]["c"], b[i]["kappa"] = shape, a, c, kap
        b[i]["n_panels"], b[i]["n_ref"], b[i]["n_theta"] = npan, nref, nth
        b[i]["theta1"], b[i]["theta2"] = 0.3 + i, 1.1 - 0.2 * i
        b[i]["cx"], b[i]["cy"], b[i]["cz"] = 3.2 * i, 0.4 * i, -0.3 * i
        b[i]["problem"] = problems[i] if problems else 0
    return sc.Scenario("edges", b, np.array(k), sc.paper_direction())


@pytest.mark.parametrize("spec", [(sc.PEANUT, 0.5, 0.3, 0.2, 8, 0, 64),
                                  (sc.CONCH, 0.5, 1.0, 0.0, 4, 2, 64)])
def test_largest_body(spec):
    s = scenario([spec, (sc.SPHERE, 0.4, 0.4, 0.0, 1, 0, 8)])
    d = geo.discretize(s)
    body = d.bodies[0]
    n = body.n
    assert n == 8192
    rows = np.array([5, 4100, 8191])
    want = oself.self_block(body, 3.0, rows=rows)
    mu = np.exp(0.003j * np.arange(d.pos.shape[0]))
    tg = np.sort(np.random.default_rng(3).choice(d.pos.shape[0], 40, replace=False))
    ps = opair.pair_sum(d, s.k, mu, targets=tg)
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        t = torch.zeros(n * n, dtype=torch.complex128, device=DEV)
        qax.qax_self_block(P.h, 0, t)
        got = t.cpu().numpy().reshape(n, n)[rows]
        scale = np.abs(want).max(axis=1, keepdims=True)
        assert (np.abs(got - want) / scale).max() < 1e-12
        del t
        v = torch.from_numpy(mu).to(DEV)
        bv = P.vec()
        qax.qax_block_apply(P.h, 0, qax.QAX_FP64, v, bv)
        back = P.vec()
        qax.qax_block_apply(P.h, 1, qax.QAX_FP64, bv, back)
        assert rel(back.cpu().numpy(), mu) < 1e-11
        qax.qax_block_apply(P.h, 1, qax.QAX_MIXED, bv, back)
        assert rel(back.cpu().numpy(), mu) < 1e-4
        out = P.vec()
        qax.qax_pair_sum(P.h, qax.QAX_FP64, v, out)
        assert rel(out.cpu().numpy()[tg], ps) < 1e-12


def test_fewest_azimuths_and_single_panel():
    s = scenario([(sc.SPHEROID, 0.5, 1.0, 0.2, 1, 0, 4), (sc.PEANUT, 0.5, 0.3, 0.1, 2, 0, 4)])
    d = geo.discretize(s)
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        for bi in (0, 1):
            body = d.bodies[bi]
            n = body.n
            rows = np.array([0, n // 2 + 1, n - 1])
            want = oself.self_block(body, 3.0, rows=rows)
            t = torch.zeros(n * n, dtype=torch.complex128, device=DEV)
            qax.qax_self_block(P.h, bi, t)
            got = t.cpu().numpy().reshape(n, n)[rows]
            assert (np.abs(got - want) / np.abs(want).max(axis=1, keepdims=True)).max() < 1e-12


def test_single_body_and_laplace_next_to_helmholtz():
    one = scenario([(sc.SPHEROID, 0.5, 1.0, 0.1, 2, 0, 16)])
    with qax.Problem(one) as P:
        out = P.vec()
        qax.qax_pair_sum(P.h, qax.QAX_FP64, torch.ones(P.N, dtype=torch.complex128, device=DEV), out)
        assert out.abs().max().item() == 0.0
        qax.qax_assemble_self(P.h)
        x = P.vec()
        info = qax.qax_solve(P.h, qax.QAX_FP64, one.dirs, x, 1, tol=1e-12, maxit=50)
        assert info["rel_res"] <= 1e-12 and info["iters"] <= 2
    two = scenario([(sc.SPHEROID, 0.5, 1.0, 0.1, 1, 0, 8), (sc.SPHERE, 0.4, 0.4, 0.0, 1, 0, 8),
                    (sc.PEANUT, 0.5, 0.3, 0.2, 1, 0, 8), (sc.SPHERE, 0.3, 0.3, 0.0, 1, 0, 8)],
                   k=(0.0, 4.0), problems=[0, 0, 1, 1])
    d = geo.discretize(two)
    mu = np.cos(0.05 * np.arange(d.pos.shape[0])) + 0.3j
    want = opair.pair_sum(d, two.k, mu)
    with qax.Problem(two) as P:
        v = torch.from_numpy(mu).to(DEV)
        out = P.vec()
        qax.qax_pair_sum(P.h, qax.QAX_FP64, v, out)
        assert rel(out.cpu().numpy(), want) < 1e-12
        qax.qax_pair_sum(P.h, qax.QAX_MIXED, v, out)
        assert rel(out.cpu().numpy(), want) < 1e-5
        assert np.abs(out.cpu().numpy() - want).max() < 1e-5 * np.abs(want).max()


def test_most_right_hand_sides():
    s = scenario([(sc.SPHEROID, 0.5, 1.0, 0.2, 1, 0, 8), (sc.PEANUT, 0.5, 0.3, 0.1, 1, 0, 8),
                  (sc.SPHERE, 0.4, 0.4, 0.0, 1, 0, 8)])
    d = geo.discretize(s)
    n = d.pos.shape[0]
    nrhs = 256
    rng = np.random.default_rng(5)
    mu = rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs))
    cols = np.array([0, 77, 255])
    want = opair.pair_sum(d, s.k, mu[:, cols])
    with qax.Problem(s) as P:
        v = torch.from_numpy(np.ascontiguousarray(mu.ravel())).to(DEV)
        out = P.vec(nrhs)
        for prec, tol in ((qax.QAX_FP64, 1e-12), (qax.QAX_MIXED, 1e-5)):
            qax.qax_pair_sum(P.h, prec, v, out, nrhs)
            assert rel(out.cpu().numpy().reshape(n, nrhs)[:, cols], want) < tol
        qax.qax_assemble_self(P.h)
        x = P.vec(nrhs)
        qax.qax_block_apply(P.h, 1, qax.QAX_MIXED, v, x, nrhs)     # matrix-core path
        y = P.vec(nrhs)
        qax.qax_block_apply(P.h, 0, qax.QAX_FP64, x, y, nrhs)
        assert rel(y.cpu().numpy(), mu.ravel()) < 1e-4
        with pytest.raises(qax.QaxError):
            qax.qax_pair_sum(P.h, qax.QAX_FP64, v, out, nrhs + 1)


@pytest.mark.parametrize("bad", [dict(n_ref=9), dict(n_ref=1, n_panels=1), dict(shape=sc.SPIRAL, kappa=0.1),
                                 dict(n_panels=8, n_ref=2, n_theta=64), dict(shape=6), dict(n_theta=66)])
def test_build_argument_errors(bad):
    s = scenario([(sc.SPHEROID, 0.5, 1.0, 0.0, 2, 0, 16)])
    for key, val in bad.items():
        s.bodies[key] = val
    h = qax.qax_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        with pytest.raises(qax.QaxError):
            qax.qax_build(h, s.bodies, s.k)
    finally:
        qax.qax_destroy(h)
