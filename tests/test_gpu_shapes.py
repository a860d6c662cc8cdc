"""The geometries of Section 6.1, Example 2 (quasi-ellipsoid, spiral, conch)
and dyadic panel refinement near the poles (N_ref of Section 6, Table 4)
through the C interface:

* nodes and area-weighted normals against the oracle (1e-13);
* self-block rows against the oracle (1e-12 of the row maximum), including
  rows in the smallest end panels, where panels two or more away are
  integrated as near panels;
* point sources inside two conches and two spirals (artificial solutions):
  the error of the refined discretisation against the unrefined one, as in
  Table 4.
"""

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import selfblock as oself
from oracle import solve as osolve
from paper_2606_31380_amd import scenarios as sc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_31380_amd import qax  # noqa: E402

DEV = torch.device("cuda", 0)


def bodies(specs, spacing=4.0):
    b = sc.make_bodies(len(specs))
    for i, (shape, a, c, kap, npan, nref, nth, t1, t2) in enumerate(specs):
        b[i]["shape"], b[i]["a"], b[i]["c"], b[i]["kappa"] = shape, a, c, kap
        b[i]["n_panels"], b[i]["n_ref"], b[i]["n_theta"] = npan, nref, nth
        b[i]["theta1"], b[i]["theta2"] = t1, t2
        b[i]["cx"], b[i]["cy"], b[i]["cz"] = spacing * i, 0.3 * i, -0.2 * i
    return b


SPECS = [(sc.SPIRAL, 0.5, 1.0, 0.0, 4, 2, 16, 0.3, 0.8),
         (sc.CONCH, 0.6, 1.0, 0.0, 3, 3, 16, 1.1, 0.4),
         (sc.QUASI_ELLIPSOID, 0.3, 1.0, 0.0, 2, 1, 16, 2.0, 1.3),
         (sc.SPHEROID, 0.5, 1.0, 0.2, 3, 2, 16, 0.7, 2.2)]


def test_nodes_match_oracle():
    s = sc.Scenario("shapes", bodies(SPECS), np.array([3.0]), sc.paper_direction())
    d = geo.discretize(s)
    with qax.Problem(s) as P:
        assert P.N == d.pos.shape[0]
        pos = torch.zeros(P.N * 3, dtype=torch.float64, device=DEV)
        aw = torch.zeros_like(pos)
        qax.qax_nodes(P.h, pos, aw)
        gp = pos.cpu().numpy().reshape(-1, 3)
        ga = aw.cpu().numpy().reshape(-1, 3)
    assert np.abs(gp - d.pos).max() < 1e-13 * np.abs(d.pos).max()
    assert np.abs(ga - d.aw).max() < 1e-13 * np.abs(d.aw).max()


@pytest.mark.parametrize("bi", [0, 1, 2, 3])
def test_self_block_rows_refined(bi):
    k = 3.0
    s = sc.Scenario("shapes", bodies(SPECS), np.array([k]), sc.paper_direction())
    d = geo.discretize(s)
    body = d.bodies[bi]
    nb = body.n
    nth = body.n_theta
    blk = 16 * nth
    rows = np.array([0, 5 * nth + 3, blk + 17, nb // 2 + 1, nb - blk + 40, nb - 1])
    want = oself.self_block(body, k, rows=rows)
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        t = torch.zeros(nb * nb, dtype=torch.complex128, device=DEV)
        qax.qax_self_block(P.h, bi, t)
        got = t.cpu().numpy().reshape(nb, nb)[rows]
    scale = np.abs(want).max(axis=1, keepdims=True)
    assert (np.abs(got - want) / scale).max() < 1e-12


def artificial_error(s):
    k = float(s.k[0])
    with qax.Problem(s) as P:
        qax.qax_assemble_self(P.h)
        pos = torch.zeros(P.N * 3, dtype=torch.float64, device=DEV)
        aw = torch.zeros_like(pos)
        qax.qax_nodes(P.h, pos, aw)
        y = pos.cpu().numpy().reshape(-1, 3)
        centres = np.stack([s.bodies["cx"], s.bodies["cy"], s.bodies["cz"]], 1)
        z = centres + np.array([0.02, -0.03, 0.05])
        b = torch.from_numpy(osolve.point_source_field(k, z, y)).to(DEV)
        mu = P.vec()
        info = qax.qax_solve_rhs(P.h, qax.QAX_FP64, b, mu, 1, tol=1e-13, maxit=500)
        assert info["rel_res"] <= 1e-13
        c = centres.mean(axis=0)
        u = np.random.default_rng(7).standard_normal((150, 3))
        pts = u / np.linalg.norm(u, axis=1)[:, None] * 8.0 + c
        out = torch.zeros(pts.shape[0], dtype=torch.complex128, device=DEV)
        qax.qax_nearfield(P.h, mu, pts, out)
        exact = osolve.point_source_field(k, z, pts)
        return float(np.linalg.norm(out.cpu().numpy() - exact) / np.linalg.norm(exact))


@pytest.mark.parametrize("shape,npan,nth,tol", [(sc.CONCH, 4, 32, 1e-10), (sc.SPIRAL, 8, 24, 1e-11)])
def test_refinement_improves_artificial_solution(shape, npan, nth, tol):
    # k = 5 as in Table 4; the spiral's centreline turns 6 times along the
    # curve, so it needs more uniform panels than the conch
    errs = {}
    for nref in (0, 4):
        spec = [(shape, 0.5, 1.0, 0.0, npan, nref, nth, 0.2, 0.9),
                (shape, 0.5, 1.0, 0.0, npan, nref, nth, 1.7, 0.3)]
        s = sc.Scenario("pair", bodies(spec, spacing=3.0), np.array([5.0]), sc.paper_direction())
        errs[nref] = artificial_error(s)
    print(shape, errs)
    assert errs[4] < tol
    assert errs[4] < 0.1 * errs[0]
