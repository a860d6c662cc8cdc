"""Pins of the oracle's geometries of Section 6.1, Example 2 (quasi-ellipsoid,
spiral, conch) and of dyadic panel refinement near the poles (the N_ref of
the notation table of Section 6; Table 4): derivatives against finite
differences, cancellation-free differences against direct ones, the
refined rule against closed-form integrals with endpoint singularities,
volumes against Cavalieri's closed forms, and Gauss's identity for the
double layer on refined bodies."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import geometry as geo
from oracle import selfblock

NEW = [geo.QUASI_ELLIPSOID, geo.SPIRAL, geo.CONCH]


@pytest.mark.parametrize("shape", NEW)
def test_curve_derivatives_finite_differences(shape):
    t = np.linspace(-1.5, 1.5, 41)
    h = 1e-5
    c0 = geo.curve(shape, 0.7, 1.0, 0.0, t)
    cp = geo.curve(shape, 0.7, 1.0, 0.0, t + h)
    cm = geo.curve(shape, 0.7, 1.0, 0.0, t - h)
    for v, d in ((0, 1), (2, 3), (4, 5), (6, 7)):
        fd = (cp[v] - cm[v]) / (2 * h)
        assert np.abs(fd - c0[d]).max() < 1e-8 * max(1.0, np.abs(c0[d]).max())


@pytest.mark.parametrize("shape", NEW)
def test_curve_differences(shape):
    rng = np.random.default_rng(3)
    t = rng.uniform(-1.5, 1.5, 60)
    dl = rng.uniform(-0.3, 0.3, 60)
    d_r, d_z, d_p, d_q = geo.curve_differences(shape, 0.7, 1.0, 0.0, t, dl)
    r0, _, z0, _, p0, _, q0, _ = geo.curve(shape, 0.7, 1.0, 0.0, t)
    r1, _, z1, _, p1, _, q1, _ = geo.curve(shape, 0.7, 1.0, 0.0, t + dl)
    assert np.allclose(d_r, r1 - r0, atol=1e-14)
    assert np.allclose(d_z, z0 - z1, atol=1e-14)
    assert np.allclose(d_p, p0 - p1, atol=1e-14)
    assert np.allclose(d_q, q0 - q1, atol=1e-14)
    # tiny offsets: full relative accuracy against 40-digit differences
    mp.mp.dps = 40
    eps = 1e-9
    e = geo.curve_differences(shape, 0.7, 1.0, 0.0, t[:12], eps)
    for i in range(12):
        tm = mp.mpf(float(t[i]))
        a0, a1 = _curve_mp(shape, mp.mpf("0.7"), tm), _curve_mp(shape, mp.mpf("0.7"), tm + mp.mpf(eps))
        want = (a1[0] - a0[0], a0[1] - a1[1], a0[2] - a1[2], a0[3] - a1[3])
        for got, w in zip((e[0][i], e[1][i], e[2][i], e[3][i]), want):
            assert abs(got - float(w)) <= 1e-12 * abs(float(w)) + 1e-300


def _curve_mp(shape, a, t):
    """r, z, p, q of the three geometries, written from the paper's
    parametrisations (Section 6.1, Example 2) in 40-digit arithmetic."""
    c, s = mp.cos(t), mp.sin(t)
    if shape == geo.QUASI_ELLIPSOID:
        return 2 * a * c, 3 * a * s, a * c, mp.mpf(0)
    if shape == geo.SPIRAL:
        return (mp.mpf("1.5") * a * c, 2 * a * s, mp.mpf("0.05") * a * mp.cos(4 * mp.pi * t),
                mp.mpf("0.1") * a * mp.sin(4 * mp.pi * t))
    f = mp.mpf("0.2") + mp.mpf("0.1") * mp.sin(8 * t)
    return a * c, mp.mpf("1.5") * a * s, a * f * c, a * f * s


def test_dyadic_panel_edges():
    e = geo.panel_edges(4, 3)
    h = math.pi / 4
    lens = np.diff(e)
    want = np.array([h / 8, h / 8, h / 4, h / 2, h, h, h / 2, h / 4, h / 8, h / 8])
    assert np.allclose(lens, want, rtol=0, atol=1e-15)
    assert e[0] == -0.5 * math.pi and e[-1] == 0.5 * math.pi
    assert np.array_equal(geo.panel_edges(5, 0), np.linspace(-0.5 * math.pi, 0.5 * math.pi, 6))


def test_refinement_resolves_endpoint_singularity():
    # int_{-pi/2}^{pi/2} sqrt(cos t) dt = sqrt(pi) Gamma(3/4) / Gamma(5/4)
    exact = math.sqrt(math.pi) * math.gamma(0.75) / math.gamma(1.25)
    errs = []
    for nref in range(6):
        d = geo.discretize_body(geo.SPHERE, 0.5, 0.5, 0.0, 4, 4, nref)
        val = np.sum(d.omega * np.sqrt(np.cos(d.t_nodes)))
        errs.append(abs(val - exact))
        # smooth integrand: exact on any panel layout
        assert abs(np.sum(d.omega * np.cos(d.t_nodes)) - 2.0) < 1e-14
    # the error sits in the end panels and scales like their length^(3/2):
    # each halving divides it by 2^(3/2)
    for e0, e1 in zip(errs[1:-1], errs[2:]):
        assert abs(e0 / e1 - 2 ** 1.5) < 0.05 * 2 ** 1.5
    assert errs[5] < 1e-2 * errs[0]


@pytest.mark.parametrize("shape,vol", [(geo.QUASI_ELLIPSOID, 16 * math.pi), (geo.SPIRAL, 6 * math.pi),
                                       (geo.CONCH, 2 * math.pi)])
def test_volume_cavalieri(shape, vol):
    # slices shifted sideways keep the volume of the (2a, 2a, 3a), (1.5a, 1.5a, 2a)
    # and (a, a, 1.5a) spheroids (a = 1)
    for nref in (0, 3):
        d = geo.discretize_body(shape, 1.0, 1.0, 0.0, 4, 32, nref)
        v = np.sum(np.sum(d.y0 * d.n0, axis=1) * d.w) / 3.0
        assert abs(v - vol) < 1e-13 * vol


@pytest.mark.parametrize("shape,npan,nref,tol", [(geo.SPIRAL, 4, 2, 1e-9), (geo.CONCH, 4, 3, 1e-11),
                                                 (geo.QUASI_ELLIPSOID, 3, 1, 1e-11)])
def test_gauss_identity_refined(shape, npan, nref, tol):
    # (1/2 + D_0)[1] = 0 on a closed surface, with panels of unequal lengths;
    # rows in the smallest panels, whose rings are close to panels two or
    # more away (those must be integrated as near panels); the spiral's
    # generating curve is singular at the poles, which limits it to ~1e-10
    nth = 32
    d = geo.discretize_body(shape, 0.5, 1.0, 0.0, npan, nth, nref)
    blk = 16 * nth
    rows = np.concatenate([np.arange(0, blk, 29), np.arange(blk, 2 * blk, 37),
                           np.arange(d.n - blk, d.n, 31), np.arange(0, d.n, 211)])
    B = selfblock.self_block(d, 0.0, rows=rows)
    assert np.abs(B @ np.ones(d.n)).max() < tol
    # the same rows with adjacent panels only as near panels fail for the
    # refined spiral and conch (the smooth rule's theta aliasing near the pole)
    if shape != geo.QUASI_ELLIPSOID:
        save = selfblock.panel_is_near
        selfblock.panel_is_near = lambda disc, pT, tT, thT, i: abs(i - pT) <= 1
        try:
            B0 = selfblock.self_block(d, 0.0, rows=rows)
        finally:
            selfblock.panel_is_near = save
        assert np.abs(B0 @ np.ones(d.n)).max() > 100 * tol
