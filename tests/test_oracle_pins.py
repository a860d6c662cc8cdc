"""Pins of the CPU oracle against quantities it does not compute itself:
closed forms, an independent arbitrary-precision library (mpmath), brute force
and invariants.  A plausible mistake anywhere in the oracle (a dropped term, a
wrong sign or index, a transposed operand) fails at least one of these."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import eval_legendre, lpmv, spherical_jn, spherical_yn

from oracle import geometry as geo
from oracle import modal, pairsum, selfblock, solve
from paper_2606_31380_amd import scenarios as sc


# ---------------------------------------------------------------- geometry
@pytest.mark.parametrize("npan,nth", [(1, 16), (2, 32)])
def test_sphere_spheroid_area_volume(npan, nth):
    # sphere: area 4 pi a^2, volume 4/3 pi a^3 (divergence theorem with x.n)
    for shape, a, c in [(geo.SPHERE, 0.5, 0.5), (geo.SPHEROID, 0.5, 1.0)]:
        d = geo.discretize_body(shape, a, c, 0.0, npan, nth)
        area = np.sum(np.linalg.norm(d.n0, axis=1) * d.w)
        vol = np.sum(np.sum(d.y0 * d.n0, axis=1) * d.w) / 3.0
        if shape == geo.SPHERE:
            area_ref = 4 * math.pi * a * a
        else:  # prolate spheroid
            e = math.sqrt(1 - a * a / (c * c))
            area_ref = 2 * math.pi * a * a * (1 + c / (a * e) * math.asin(e))
        vol_ref = 4.0 / 3.0 * math.pi * a * a * c
        tol = 1e-9 if npan == 1 else 1e-13
        assert abs(area - area_ref) < tol * area_ref
        assert abs(vol - vol_ref) < tol * vol_ref
        # closed surface: sum of area normals vanishes
        assert np.abs((d.n0 * d.w[:, None]).sum(axis=0)).max() < 1e-13


def test_bent_volume_cavalieri_and_outward():
    # horizontal slices shifted sideways keep the volume (Cavalieri); normals outward
    for shape, a, c in [(geo.SPHEROID, 0.5, 1.0), (geo.PEANUT, 0.5, 0.3)]:
        d0 = geo.discretize_body(shape, a, c, 0.0, 2, 32)
        d1 = geo.discretize_body(shape, a, c, 0.3, 2, 32)
        v0 = np.sum(np.sum(d0.y0 * d0.n0, axis=1) * d0.w) / 3.0
        v1 = np.sum(np.sum(d1.y0 * d1.n0, axis=1) * d1.w) / 3.0
        assert abs(v0 - v1) < 1e-12 * v0
        assert v0 > 0
        # the rotated world-frame copy has the same volume about its centre
        s = sc.tiny(n_bodies=1, n_panels=2, n_theta=32, shapes=(shape,))
        s.bodies["kappa"] = 0.3
        dw = geo.discretize(s)
        cen = dw.centres[0]
        vw = np.sum(np.sum((dw.pos - cen) * dw.aw, axis=1)) / 3.0
        assert abs(vw - v1) < 1e-12 * v1


@pytest.mark.parametrize("c", [0.3, -0.2])
def test_peanut_closed_forms(c):
    # peanut of revolution, polar radius rho(psi) = a (1 + c cos 2 psi) with psi
    # the polar angle: waist a (1 - c) at the equator, a (1 + c) at the poles;
    # volume (2 pi / 3) int_0^pi rho^3 sin psi dpsi = (2 pi / 3) a^3 int_-1^1
    # (A + B u^2)^3 du with A = 1 - c, B = 2 c (u = cos psi), a polynomial;
    # area 2 pi int rho sin psi sqrt(rho^2 + rho'^2) dpsi by mpmath quadrature
    a = 0.5
    r, _, z, _, _, _, _, _ = geo.curve(geo.PEANUT, a, c, 0.0, np.array([0.0, 0.5 * math.pi, -0.5 * math.pi]))
    assert abs(r[0] - a * (1 - c)) < 1e-15 and abs(z[0]) < 1e-15
    assert abs(z[1] - a * (1 + c)) < 1e-15 and abs(z[2] + a * (1 + c)) < 1e-15
    A, B = 1.0 - c, 2.0 * c
    vol_ref = 2.0 * math.pi / 3.0 * a ** 3 * (2 * A ** 3 + 2 * A * A * B + 1.2 * A * B * B + 2.0 / 7.0 * B ** 3)
    rho = lambda ps: a * (1 + c * mp.cos(2 * ps))
    drho = lambda ps: -2 * a * c * mp.sin(2 * ps)
    area_ref = float(2 * mp.pi * mp.quad(lambda ps: rho(ps) * mp.sin(ps) * mp.sqrt(rho(ps) ** 2 + drho(ps) ** 2),
                                         [0, mp.pi / 2, mp.pi]))
    d = geo.discretize_body(geo.PEANUT, a, c, 0.0, 4, 32)
    area = np.sum(np.linalg.norm(d.n0, axis=1) * d.w)
    vol = np.sum(np.sum(d.y0 * d.n0, axis=1) * d.w) / 3.0
    assert abs(vol - vol_ref) < 1e-12 * vol_ref, (vol, vol_ref)
    assert abs(area - area_ref) < 1e-12 * area_ref, (area, area_ref)


def test_curve_differences_match_direct():
    rng = np.random.default_rng(1)
    for shape, a, c in [(geo.SPHERE, 0.5, 0.5), (geo.SPHEROID, 0.5, 1.0), (geo.PEANUT, 0.5, 0.3)]:
        t = rng.uniform(-1.5, 1.5, 50)
        dl = rng.uniform(-0.3, 0.3, 50)
        d_r, d_z, d_p, _ = geo.curve_differences(shape, a, c, 0.27, t, dl)
        r0, _, z0, _, p0, _, _, _ = geo.curve(shape, a, c, 0.27, t)
        r1, _, z1, _, p1, _, _, _ = geo.curve(shape, a, c, 0.27, t + dl)
        assert np.allclose(d_r, r1 - r0, atol=1e-14)
        assert np.allclose(d_z, z0 - z1, atol=1e-14)
        assert np.allclose(d_p, p0 - p1, atol=1e-14)


# ---------------------------------------------------------------- special functions
def test_elliptic_agm_closed_forms():
    k = np.array([1 / math.sqrt(2)])
    K, E = modal.ellipke(k, np.sqrt(1 - k * k))
    g = math.gamma(0.25)
    assert abs(K[0] - g * g / (4 * math.sqrt(math.pi))) < 1e-15
    assert abs(E[0] - (g * g / (8 * math.sqrt(math.pi)) + math.pi ** 1.5 / (g * g))) < 1e-15
    kk = np.array([0.1, 0.5, 0.9, 0.999999])
    K, E = modal.ellipke(kk, np.sqrt(1 - kk * kk))
    for i, kv in enumerate(kk):
        assert abs(K[i] - float(mp.ellipk(kv * kv))) < 2e-15 * K[i]
        assert abs(E[i] - float(mp.ellipe(kv * kv))) < 2e-15 * E[i]


@pytest.mark.parametrize("chi", [1.0 + 1e-10, 1.0001, 1.01, 1.5, 3.0, 40.0])
def test_toroidal_q_vs_mpmath(chi):
    mp.mp.dps = 40
    Q, Qp = modal.toroidal_q(np.array([chi]), np.array([chi - 1.0]), 40)
    for m in (0, 1, 2, 7, 20, 40):
        ref = float(mp.re(mp.legenq(m - 0.5, 0, mp.mpf(chi), type=3)))
        assert abs(Q[0, m] - ref) <= 3e-14 * abs(ref)
        dref = float(mp.re(mp.diff(lambda x: mp.legenq(m - 0.5, 0, x, type=3), mp.mpf(chi))))
        assert abs(Qp[0, m] - dref) <= 1e-11 * abs(dref)


def _mp_modes(k, r, rt, c, m, which):
    mp.mp.dps = 30

    def f(phi):
        rho = mp.sqrt((r - rt) ** 2 + c ** 2 + 4 * r * rt * mp.sin(phi / 2) ** 2)
        if which == "G":
            v = mp.exp(1j * k * rho) / (4 * mp.pi * rho)
        else:
            d = mp.exp(1j * k * rho) * (1j * k * rho - 1) / (4 * mp.pi * rho ** 3)
            v = d * (r - rt * mp.cos(phi)) if which == "A" else d * (-c)
        return v * mp.cos(m * phi)

    return complex(2 * mp.quad(f, [0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1, mp.pi]))


@pytest.mark.parametrize("geom", [(1.0, 1.0, 0.1), (0.5, 0.45, 0.02), (0.3, 0.3002, 1e-4)])
@pytest.mark.parametrize("k", [0.0, 2.0, 10.0])
def test_modal_green_vs_azimuthal_quadrature(geom, k):
    r, rt, c = (np.array([v]) for v in geom)
    chim1 = ((r - rt) ** 2 + c * c) / (2 * r * rt)
    A, B = modal.derivative_modes(k, r, rt, c, 1 + chim1, chim1, 5)
    G = modal.helmholtz_g_modes(k, r, rt, c, 1 + chim1, chim1, 5)
    for m in (0, 1, 4):
        for arr, w in ((G, "G"), (A, "A"), (B, "B")):
            ref = _mp_modes(k, *geom, m, w)
            assert abs(arr[0, m] - ref) <= 1e-12 * abs(ref), (w, m)


def test_gj_modal_equals_direct_route():
    # both azimuthal routes agree where both are valid (chi - 1 around 0.1)
    d = geo.discretize_body(geo.PEANUT, 0.5, 0.3, 0.25, 2, 16)
    N = 8
    t_t = np.full(6, d.t_nodes[5])
    th_t = d.theta[[0, 3, 5, 7, 9, 12]]
    dl = np.array([0.15, -0.2, 0.25, 0.18, -0.3, 0.22])
    loc = modal.local_frame_rel(d.shape, d.a, d.c, d.kappa, t_t, th_t, dl)
    assert np.all((loc["chim1"] > 0.01) & (loc["chim1"] < 1.0))
    for k in (0.0, 3.0):
        gm = modal.gj_modal(k, N, loc, L=256)
        x, _ = geo.surface_point_normal(d.shape, d.a, d.c, d.kappa, t_t, th_t)
        gd = modal.gj_direct(k, N, x, selfblock.slice_geometry(d, t_t + dl), L=2048)
        assert np.abs(gm - gd).max() < 1e-12 * np.abs(gd).max()


# ---------------------------------------------------------------- self block
@pytest.mark.parametrize("shape,a,c,kap,npan", [(geo.SPHEROID, 0.5, 1.0, 0.3, 1),
                                                 (geo.PEANUT, 0.5, 0.3, 0.2, 2),
                                                 (geo.SPHEROID, 0.5, 1.0, 0.25, 3)])
def test_gauss_identity_self_block(shape, a, c, kap, npan):
    # (1/2 + D_0)[1] = 0 on any closed surface (exterior limit of Gauss's integral)
    d = geo.discretize_body(shape, a, c, kap, npan, 16)
    rows = np.arange(0, d.n, 11)
    B = selfblock.self_block(d, 0.0, rows=rows)
    assert np.abs(B @ np.ones(d.n)).max() < 1e-12


def _sphere_lambda(n, ka):
    h = spherical_jn(n, ka) + 1j * spherical_yn(n, ka)
    return 1j * ka * ka * spherical_jn(n, ka, derivative=True) * h


def test_sphere_double_layer_eigenvalues():
    # (1/2 + D) Y_n^m = lambda_n Y_n^m, lambda_n = i (ka)^2 j_n'(ka) h_n(ka)
    a, k = 1.0, 1.0
    d = geo.discretize_body(geo.SPHERE, a, a, 0.0, 2, 16)
    rows = np.arange(0, d.n, 9)
    B = selfblock.self_block(d, k, rows=rows)
    cosg = d.y0[:, 2] / a
    phi = np.arctan2(d.y0[:, 1], d.y0[:, 0])
    for n, m in [(0, 0), (1, 0), (2, 0), (3, 0), (2, 1), (3, 2), (3, 3)]:
        mu = lpmv(m, n, cosg) * np.cos(m * phi)
        lam = _sphere_lambda(n, k * a)
        assert np.abs(B @ mu - lam * mu[rows]).max() < 1e-11, (n, m)


def test_self_block_k10_against_eigenvalues():
    a, k = 0.5, 10.0
    d = geo.discretize_body(geo.SPHERE, a, a, 0.0, 3, 32)
    rows = np.arange(3, d.n, 97)
    B = selfblock.self_block(d, k, rows=rows)
    cosg = d.y0[:, 2] / a
    for n in (0, 2, 5):
        mu = eval_legendre(n, cosg)
        assert np.abs(B @ mu - _sphere_lambda(n, k * a) * mu[rows]).max() < 1e-9


# ---------------------------------------------------------------- pair sum
def test_pair_sum_brute_force():
    s = sc.tiny(n_bodies=3, n_panels=1, n_theta=4, k=3.0, shapes=(geo.SPHEROID, geo.PEANUT))
    d = geo.discretize(s)
    rng = np.random.default_rng(0)
    mu = rng.standard_normal(d.pos.shape[0]) + 1j * rng.standard_normal(d.pos.shape[0])
    ref = pairsum.pair_sum_bruteforce(d, s.k, mu)
    out = pairsum.pair_sum(d, s.k, mu, chunk=17)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


def test_pair_sum_multi_problem_brute_force():
    s = sc.tiny(n_bodies=4, n_panels=1, n_theta=4, k=2.0)
    s.bodies["problem"] = [0, 1, 0, 1]
    s.k = np.array([2.0, 5.0])
    d = geo.discretize(s)
    mu = np.linspace(0.1, 1.0, d.pos.shape[0]) * (1 + 0.5j)
    ref = pairsum.pair_sum_bruteforce(d, s.k, mu)
    assert np.abs(pairsum.pair_sum(d, s.k, mu) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_pair_sum_exterior_sphere_closed_form():
    # the inter-body smooth rule reproduces the exterior double-layer potential
    # of a sphere: D[P_n](x) = i k^2 a^2 j_n'(ka) h_n(k|x|) P_n(cos psi_x)
    s = sc.two_spheres(n_panels=2, n_theta=32, k=2.0)
    s.bodies["cx"] = [-1.5, 1.5]
    d = geo.discretize(s)
    a, k = 0.5, 2.0
    n0 = d.offsets[1]
    src_local = d.pos[:n0] - d.centres[0]
    for n in (0, 1, 3):
        mu = np.zeros(d.pos.shape[0], dtype=np.complex128)
        mu[:n0] = eval_legendre(n, src_local[:, 2] / a)
        tgt = np.arange(n0, d.pos.shape[0], 13)
        out = pairsum.pair_sum(d, s.k, mu, targets=tgt)
        x = d.pos[tgt] - d.centres[0]
        rx = np.linalg.norm(x, axis=1)
        h = spherical_jn(n, k * rx) + 1j * spherical_yn(n, k * rx)
        ref = 1j * k * k * a * a * spherical_jn(n, k * a, derivative=True) * h * eval_legendre(n, x[:, 2] / rx)
        assert np.abs(out - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_near_field_exterior_sphere_closed_form():
    # D[P_n](x) at points off the sphere, as the pair sum at nodes above
    s = sc.single_sphere(0.5, 2, 32, 2.0)
    d = geo.discretize(s)
    a, k = 0.5, 2.0
    rng = np.random.default_rng(4)
    u = rng.standard_normal((40, 3))
    pts = u / np.linalg.norm(u, axis=1)[:, None] * rng.uniform(1.2, 4.0, (40, 1)) + d.centres[0]
    loc = d.pos - d.centres[0]
    for n in (0, 2, 5):
        mu = eval_legendre(n, loc[:, 2] / a).astype(np.complex128)
        out = solve.near_field(d, s.k, mu, pts)
        x = pts - d.centres[0]
        rx = np.linalg.norm(x, axis=1)
        h = spherical_jn(n, k * rx) + 1j * spherical_yn(n, k * rx)
        ref = 1j * k * k * a * a * spherical_jn(n, k * a, derivative=True) * h * eval_legendre(n, x[:, 2] / rx)
        assert np.abs(out - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())


def test_artificial_point_source_solution():
    # exterior Dirichlet data of a point source inside each body: the solved
    # double-layer density reproduces the source field outside and its far
    # field (end to end: self blocks, pair sums, near and far field)
    s = sc.tiny(n_bodies=2, n_panels=2, n_theta=16, k=2.0, spacing=2.5)
    s.bodies["kappa"] = 0.2            # congruent bodies (different rotations): one self block
    d = geo.discretize(s)
    z = d.centres + np.array([0.05, -0.03, 0.1])
    b = solve.point_source_field(2.0, z, d.pos)
    blk = solve.self_blocks(d, s.k, body_ids=[0])[0]
    blocks = {0: blk, 1: blk}
    mu = np.linalg.solve(solve.dense_matrix_fast(d, s.k, blocks), b)
    rng = np.random.default_rng(5)
    u = rng.standard_normal((30, 3))
    pts = u / np.linalg.norm(u, axis=1)[:, None] * 6.0 + d.centres.mean(axis=0)
    err = solve.near_field(d, s.k, mu, pts) - solve.point_source_field(2.0, z, pts)
    assert np.abs(err).max() < 1e-8 * np.abs(solve.point_source_field(2.0, z, pts)).max()
    xhat = u / np.linalg.norm(u, axis=1)[:, None]
    ff = solve.far_field(d, s.k, mu, xhat)
    assert np.abs(ff - solve.point_source_far_field(2.0, z, xhat)).max() < 1e-8


def test_pair_sum_rigid_motion_invariance():
    s = sc.tiny(n_bodies=3, n_panels=1, n_theta=8, k=4.0)
    d1 = geo.discretize(s)
    R = geo.rotation(0.7, 1.9)
    s2 = sc.tiny(n_bodies=3, n_panels=1, n_theta=8, k=4.0)
    # rotate + translate every body as a whole: compose rotations and move centres
    mu = np.cos(np.arange(d1.pos.shape[0]) * 0.37) + 0.2j
    out1 = pairsum.pair_sum(d1, s.k, mu)
    d2 = geo.discretize(s2)
    d2.pos = d1.pos @ R.T + np.array([3.0, -1.0, 2.0])
    d2.aw = d1.aw @ R.T
    out2 = pairsum.pair_sum(d2, s.k, mu)
    assert np.abs(out1 - out2).max() < 1e-12 * np.abs(out1).max()


# ---------------------------------------------------------------- solve
def _mie_far(k, a, gammas, nmax=40):
    out = np.zeros(len(gammas), dtype=np.complex128)
    for n in range(nmax):
        h = spherical_jn(n, k * a) + 1j * spherical_yn(n, k * a)
        out += (2 * n + 1) * spherical_jn(n, k * a) / h * eval_legendre(n, np.cos(gammas))
    return 1j / k * out


def test_mie_sound_soft_sphere():
    s = sc.single_sphere(0.5, 2, 16, 2.0)
    d = geo.discretize(s)
    blocks = solve.self_blocks(d, s.k)
    b = solve.rhs_planewave(d, s.k, s.dirs)[:, 0]
    mu, _, _ = solve.solve(d, s.k, blocks, b, method="dense")
    g = np.array([0.0, 0.7, math.pi / 2, 2.5, math.pi])
    xh = np.stack([np.sin(g), 0 * g, np.cos(g)], axis=1)
    u = solve.far_field(d, s.k, mu, xh)
    assert np.abs(u - _mie_far(2.0, 0.5, g)).max() < 1e-10


# ---------------------------------------------------------------- combined field
def _axisym_block(body, k, kind="dl"):
    """Full self block of an axisymmetric body (kappa = 0) from its rows at
    azimuth 0: rotating the target by theta_j shifts every column's azimuth."""
    nth = body.n_theta
    rows0 = np.arange(0, body.n, nth)
    B0 = selfblock.self_block(body, k, rows=rows0, kind=kind)       # (n / nth, n)
    nrow = rows0.shape[0]
    out = np.zeros((body.n, body.n), dtype=np.complex128)
    cols = np.arange(body.n)
    base, cj = cols - cols % nth, cols % nth
    for j in range(nth):
        out[j::nth, :] = B0[:, base + (cj - j) % nth]
    assert out.shape[0] == nrow * nth
    return out


def test_axisymmetric_block_expansion():
    # the shift rule used below against directly computed rows
    body = geo.discretize(sc.single_sphere(0.5, 1, 8, 2.0)).bodies[0]
    full = _axisym_block(body, 2.0, kind="sl")
    rows = np.array([3, 21, 77])
    assert np.abs(full[rows] - selfblock.self_block(body, 2.0, rows=rows, kind="sl")).max() < 1e-13


def test_sphere_single_layer_eigenvalues():
    # S[P_n] = i k a^2 j_n(ka) h_n(ka) P_n on a sphere (zonal harmonics)
    a, k = 0.5, 2.0
    d = geo.discretize(sc.single_sphere(a, 2, 16, k))
    body = d.bodies[0]
    rows = np.arange(0, body.n, 29)
    S = selfblock.self_block(body, k, rows=rows, kind="sl")
    for n in range(4):
        v = eval_legendre(n, body.y0[:, 2] / a)
        lam = 1j * k * a * a * spherical_jn(n, k * a) * (spherical_jn(n, k * a) + 1j * spherical_yn(n, k * a))
        assert np.abs(S @ v - lam * v[rows]).max() < 1e-10 * np.abs(lam * v[rows]).max()


def _interior_neumann_k(a=0.5):
    # first zero of j_1' (an interior Neumann eigenvalue of the sphere)
    from scipy.optimize import brentq
    return brentq(lambda x: spherical_jn(1, x, derivative=True), 1.5, 2.5) / a


def test_combined_field_mie_and_interior_resonance():
    # at an interior Neumann eigenvalue the double-layer system is singular
    # (its n = 1 eigenvalue i (ka)^2 j_1'(ka) h_1(ka) vanishes); the combined
    # field D - i eta S still reproduces the Mie far field
    a = 0.5
    k = _interior_neumann_k(a)
    s = sc.single_sphere(a, 2, 16, k)
    d = geo.discretize(s)
    b = solve.rhs_planewave(d, s.k, s.dirs)[:, 0]
    g = np.array([0.0, 0.7, math.pi / 2, 2.5, math.pi])
    xh = np.stack([np.sin(g), 0 * g, np.cos(g)], axis=1)
    D = _axisym_block(d.bodies[0], k)
    cf = D - 1j * k * _axisym_block(d.bodies[0], k, kind="sl")
    bl = {0: cf}
    mu, _, _ = solve.solve(d, s.k, bl, b, method="dense", eta=k)
    u = solve.far_field(d, s.k, mu, xh, eta=k)
    assert np.abs(u - _mie_far(k, a, g)).max() < 1e-9
    sv = np.linalg.svd(D, compute_uv=False)
    svc = np.linalg.svd(cf, compute_uv=False)
    assert sv.min() < 1e-6 * sv.max() and svc.min() > 0.05 * svc.max()


def test_combined_field_artificial_solution():
    s = sc.tiny(n_bodies=2, n_panels=2, n_theta=16, k=2.0, spacing=2.5)
    s.bodies["kappa"] = 0.0            # axisymmetric (rotated) spheroids: blocks by shifts
    d = geo.discretize(s)
    eta = 2.0
    z = d.centres + np.array([0.05, -0.03, 0.1])
    b = solve.point_source_field(2.0, z, d.pos)
    blk = _axisym_block(d.bodies[0], 2.0) - 1j * eta * _axisym_block(d.bodies[0], 2.0, kind="sl")
    rows = np.array([5, 300])           # the shortcut against direct rows of the combined block
    assert np.abs(blk[rows] - selfblock.self_block_cf(d.bodies[0], 2.0, eta, rows=rows)).max() < 1e-12
    mu = np.linalg.solve(solve.dense_matrix_fast(d, s.k, {0: blk, 1: blk}, eta=eta), b)
    rng = np.random.default_rng(5)
    u = rng.standard_normal((30, 3))
    xhat = u / np.linalg.norm(u, axis=1)[:, None]
    pts = xhat * 6.0 + d.centres.mean(axis=0)
    exact = solve.point_source_field(2.0, z, pts)
    assert np.abs(solve.near_field(d, s.k, mu, pts, eta=eta) - exact).max() < 1e-8 * np.abs(exact).max()
    ff = solve.far_field(d, s.k, mu, xhat, eta=eta)
    assert np.abs(ff - solve.point_source_far_field(2.0, z, xhat)).max() < 1e-8


def test_single_layer_first_kind_mie():
    # S mu = -u_inc on a sphere (k a = 1, away from interior Dirichlet
    # eigenvalues) reproduces the Mie far field of the sound-soft sphere
    a, k = 0.5, 2.0
    s = sc.single_sphere(a, 2, 16, k)
    d = geo.discretize(s)
    b = solve.rhs_planewave(d, s.k, s.dirs)[:, 0]
    S = _axisym_block(d.bodies[0], k, kind="sl")
    mu, _, _ = solve.solve(d, s.k, {0: S}, b, method="dense", single=True)
    g = np.array([0.0, 0.7, math.pi / 2, 2.5, math.pi])
    xh = np.stack([np.sin(g), 0 * g, np.cos(g)], axis=1)
    assert np.abs(solve.far_field(d, s.k, mu, xh, single=True) - _mie_far(k, a, g)).max() < 1e-10


def test_single_layer_artificial_solution_and_brute_force():
    s = sc.tiny(n_bodies=2, n_panels=2, n_theta=16, k=2.0, spacing=2.5)
    s.bodies["kappa"] = 0.0
    d = geo.discretize(s)
    z = d.centres + np.array([0.05, -0.03, 0.1])
    b = solve.point_source_field(2.0, z, d.pos)
    S = _axisym_block(d.bodies[0], 2.0, kind="sl")
    mu = np.linalg.solve(solve.dense_matrix_fast(d, s.k, {0: S, 1: S}, single=True), b)
    rng = np.random.default_rng(6)
    u = rng.standard_normal((30, 3))
    xhat = u / np.linalg.norm(u, axis=1)[:, None]
    pts = xhat * 6.0 + d.centres.mean(axis=0)
    exact = solve.point_source_field(2.0, z, pts)
    assert np.abs(solve.near_field(d, s.k, mu, pts, single=True) - exact).max() < 1e-8 * np.abs(exact).max()
    ff = solve.far_field(d, s.k, mu, xhat, single=True)
    assert np.abs(ff - solve.point_source_far_field(2.0, z, xhat)).max() < 1e-8
    # the single-layer pair sum against a plain double loop
    t = sc.tiny(n_bodies=3, n_panels=1, n_theta=8, k=3.0)
    dt = geo.discretize(t)
    m = np.cos(np.arange(dt.pos.shape[0]) * 0.7) - 0.2j
    out = pairsum.pair_sum(dt, t.k, m, single=True)
    ref = np.zeros_like(out)
    for i in range(dt.pos.shape[0]):
        for j in range(dt.pos.shape[0]):
            if dt.body[i] != dt.body[j]:
                r = math.sqrt(float((dt.pos[j] - dt.pos[i]) @ (dt.pos[j] - dt.pos[i])))
                ref[i] += complex(math.cos(3.0 * r), math.sin(3.0 * r)) / (4 * math.pi * r) \
                    * math.sqrt(float(dt.aw[j] @ dt.aw[j])) * m[j]
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()


def test_combined_pair_sum_brute_force():
    s = sc.tiny(n_bodies=3, n_panels=1, n_theta=8, k=3.0)
    d = geo.discretize(s)
    mu = np.cos(np.arange(d.pos.shape[0]) * 0.3) + 0.4j
    eta = 1.7
    out = pairsum.pair_sum(d, s.k, mu, eta=eta)
    ref = np.zeros_like(out)
    for i in range(d.pos.shape[0]):
        for j in range(d.pos.shape[0]):
            if d.body[i] == d.body[j]:
                continue
            dx = d.pos[j] - d.pos[i]
            r = math.sqrt(float(dx @ dx))
            g = complex(math.cos(3.0 * r), math.sin(3.0 * r)) / (4 * math.pi * r)
            dl = g * (1j * 3.0 * r - 1.0) / (r * r) * float(d.aw[j] @ dx)
            ref[i] += (dl - 1j * eta * g * math.sqrt(float(d.aw[j] @ d.aw[j]))) * mu[j]
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.fixture(scope="module")
def two_body():
    s = sc.tiny(n_bodies=2, n_panels=1, n_theta=12, k=2.0, spacing=2.5)
    d = geo.discretize(s)
    blocks = solve.self_blocks(d, s.k)
    return s, d, blocks


def test_gmres_matches_dense(two_body):
    s, d, blocks = two_body
    b = solve.rhs_planewave(d, s.k, s.dirs)[:, 0]
    x_dense, _, _ = solve.solve(d, s.k, blocks, b, method="dense")
    x_g, its, _ = solve.solve(d, s.k, blocks, b, method="gmres", tol=1e-13)
    assert its > 2
    assert np.linalg.norm(x_g - x_dense) < 1e-11 * np.linalg.norm(x_dense)
    A = solve.dense_matrix_fast(d, s.k, blocks)
    A2 = solve.dense_matrix(d, s.k, blocks)
    assert np.abs(A - A2).max() < 1e-14 * np.abs(A).max()


def test_far_field_reciprocity(two_body):
    # u_inf(xhat; d) = u_inf(-d; -xhat) for the exact solution (holds to
    # discretisation accuracy for the Nystrom solution)
    s, d, blocks = two_body
    A = solve.dense_matrix_fast(d, s.k, blocks)
    rng = np.random.default_rng(3)
    for _ in range(3):
        u = rng.standard_normal((2, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        dvec, xh = u[0], u[1]
        mu1 = np.linalg.solve(A, solve.rhs_planewave(d, s.k, dvec[None])[:, 0])
        mu2 = np.linalg.solve(A, solve.rhs_planewave(d, s.k, -xh[None])[:, 0])
        f1 = solve.far_field(d, s.k, mu1, xh[None])[0]
        f2 = solve.far_field(d, s.k, mu2, -dvec[None])[0]
        assert abs(f1 - f2) < 1e-6 * max(abs(f1), 1e-3)
