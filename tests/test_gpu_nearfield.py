"""Near-field evaluation and the artificial point-source solutions through the
C interface.

* qax_nearfield against the oracle's direct sum (FP64, 1e-12), for one and
  two right-hand sides and for the second of two independent problems;
* end to end: the boundary values of point sources placed inside the bodies
  (qax_solve_rhs) give a density whose near field and far field reproduce the
  exact source field (the error measure of the paper's numerical section),
  with spectral improvement under refinement;
* argument errors.
"""
import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import solve as osolve
from paper_2606_31380_amd import scenarios as sc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_31380_amd import qax  # noqa: E402

DEV = torch.device("cuda", 0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def shell_points(n, centre, radius, seed):
    u = np.random.default_rng(seed).standard_normal((n, 3))
    return u / np.linalg.norm(u, axis=1)[:, None] * radius + centre


def lattice(n_panels, n_theta, k=3.0, n_side=2, spacing=3.0, problem=0, shift=0.0):
    rng = np.random.default_rng(8)
    nb = n_side ** 3
    b = sc.make_bodies(nb)
    i = 0
    for x in range(n_side):
        for y in range(n_side):
            for z in range(n_side):
                b[i]["shape"], b[i]["a"], b[i]["c"] = sc.SPHEROID, 0.5, 1.0
                b[i]["kappa"] = (0.1, 0.25)[i % 2]
                b[i]["n_panels"], b[i]["n_theta"] = n_panels, n_theta
                b[i]["theta1"], b[i]["theta2"] = rng.uniform(0, 2 * math.pi, 2)
                b[i]["cx"], b[i]["cy"], b[i]["cz"] = spacing * x + shift, spacing * y, spacing * z
                b[i]["problem"] = problem
                i += 1
    return sc.Scenario("lattice", b, np.array([k]), sc.paper_direction())


def test_nearfield_matches_oracle():
    s = lattice(1, 12)
    d = geo.discretize(s)
    n = d.pos.shape[0]
    rng = np.random.default_rng(1)
    mu = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    c = d.centres.mean(axis=0)
    # far shell and points between the bodies (distance >= 1 from the surfaces)
    pts = np.concatenate([shell_points(300, c, 9.0, 2), c + rng.uniform(-0.3, 0.3, (20, 3))])
    want = osolve.near_field(d, s.k, mu, pts)
    with qax.Problem(s) as P:
        u = torch.zeros(pts.shape[0] * 2, dtype=torch.complex128, device=DEV)
        qax.qax_nearfield(P.h, torch.from_numpy(np.ascontiguousarray(mu.ravel())).to(DEV), pts, u, nrhs=2)
        assert rel(u.cpu().numpy().reshape(-1, 2), want) < 1e-12
        u1 = torch.zeros(pts.shape[0], dtype=torch.complex128, device=DEV)
        qax.qax_nearfield(P.h, torch.from_numpy(np.ascontiguousarray(mu[:, 1])).to(DEV), pts, u1)
        assert rel(u1.cpu().numpy(), want[:, 1]) < 1e-12


def test_nearfield_second_problem():
    a = lattice(1, 12, k=2.0)
    b = lattice(1, 10, k=4.5, problem=1, shift=0.4)
    s = sc.Scenario("two", np.concatenate([a.bodies, b.bodies]), np.array([2.0, 4.5]), a.dirs)
    d = geo.discretize(s)
    n = d.pos.shape[0]
    mu = np.exp(0.013j * np.arange(n)) * (1 + 0.1 * np.cos(np.arange(n)))
    pts = shell_points(200, d.centres.mean(axis=0), 10.0, 3)
    want = osolve.near_field(d, s.k, mu, pts, problem=1)
    with qax.Problem(s) as P:
        u = torch.zeros(pts.shape[0], dtype=torch.complex128, device=DEV)
        qax.qax_nearfield(P.h, torch.from_numpy(mu).to(DEV), pts, u, problem=1)
        assert rel(u.cpu().numpy(), want) < 1e-12


def artificial_error(s, prec=qax.QAX_FP64, tol=1e-12):
    """Solve with the boundary values of point sources inside the bodies and
    return the relative near-field and far-field errors."""
    k = float(s.k[0])
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        pos = torch.zeros(P.N * 3, dtype=torch.float64, device=DEV)
        aw = torch.zeros_like(pos)
        qax.qax_nodes(P.h, pos, aw)
        y = pos.cpu().numpy().reshape(-1, 3)
        centres = np.stack([s.bodies["cx"], s.bodies["cy"], s.bodies["cz"]], 1)
        z = centres + np.array([0.04, -0.03, 0.08])
        b = torch.from_numpy(osolve.point_source_field(k, z, y)).to(DEV)
        mu = P.vec()
        info = qax.qax_solve_rhs(P.h, prec, b, mu, 1, tol=tol, maxit=500)
        assert info["rel_res"] <= tol
        c = centres.mean(axis=0)
        pts = shell_points(200, c, np.abs(centres - c).max() + 6.0, 7)
        u = torch.zeros(pts.shape[0], dtype=torch.complex128, device=DEV)
        qax.qax_nearfield(P.h, mu, pts, u)
        exact = osolve.point_source_field(k, z, pts)
        xhat = (pts - c) / np.linalg.norm(pts - c, axis=1)[:, None]
        ff = torch.zeros(xhat.shape[0], dtype=torch.complex128, device=DEV)
        qax.qax_farfield(P.h, mu, xhat, ff)
        ff_exact = osolve.point_source_far_field(k, z, xhat)
        return rel(u.cpu().numpy(), exact), rel(ff.cpu().numpy(), ff_exact)


def test_artificial_solution_spectral_convergence():
    e_coarse, _ = artificial_error(lattice(1, 16))
    e_fine, f_fine = artificial_error(lattice(2, 32))
    # 16 GL nodes per body in s (one panel) limit the coarse case to ~3e-5;
    # two panels reach ~2e-11
    assert e_fine < 1e-10 and f_fine < 1e-10
    assert e_fine < 1e-4 * e_coarse


def test_artificial_solution_bench_lattice():
    # the benchmark's 27 bent spheroids (32 GL x 64 azimuths, k = 5)
    s = sc.lattice27()
    e64, f64 = artificial_error(s)
    assert e64 < 1e-10 and f64 < 1e-10
    em, fm = artificial_error(s, prec=qax.QAX_MIXED, tol=1e-8)
    assert em < 2e-8 and fm < 2e-8


def test_nearfield_argument_errors():
    s = lattice(1, 8)
    with qax.Problem(s) as P:
        mu = P.vec()
        u = torch.zeros(4, dtype=torch.complex128, device=DEV)
        with pytest.raises(qax.QaxError):
            qax.qax_nearfield(P.h, mu, np.zeros((4, 3)), u, problem=1)
        with pytest.raises(qax.QaxError):
            qax.qax_nearfield(P.h, mu, np.array([[0.0, 0.0, np.nan]] * 4), u)
        qax.qax_assemble_self(P.h)
        with pytest.raises(qax.QaxError):
            qax.qax_solve_rhs(P.h, qax.QAX_FP64, mu, mu, 1)
