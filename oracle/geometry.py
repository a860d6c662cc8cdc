"""Oracle geometry: quasi-axisymmetric surfaces and their Nystrom nodes.

Surface (Section 2, equation para_quasi):
    y(s, theta) = (r(s) cos theta + p(s), r(s) sin theta + q(s), z(s)).
Tangents d_s, d_theta and Jacobian |J| = |d_s x d_theta| (Section 3.1,
equation smu).  Nodes: N_P panels x 16 Gauss-Legendre nodes in s and
theta_j = j pi / N, j = 0..2N-1 (Section 3.1).  Smooth-rule weight
|J| (pi/N) omega_il (Section 3.1, equation sx).  Rigid motion
x = R x0 + c, n = R n0 with R = Rz(theta1) Ry(theta2) (Section 6.2, Example 5).

Readings (the paper is silent): the generating curve runs south to north with
s = t in [-pi/2, pi/2]; the outward area normal is d_theta x d_s; the bent axis
is the circle of radius 1/kappa tangent to the z-axis at the origin,
p = kappa z^2 / (1 + sqrt(1 - kappa^2 z^2)), q = 0; panels are uniform in t.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GL_ORDER = 16
SPHERE, SPHEROID, PEANUT = 0, 1, 2
QUASI_ELLIPSOID, SPIRAL, CONCH = 3, 4, 5
T0, T1 = -0.5 * math.pi, 0.5 * math.pi


def gauss_legendre(n: int):
    """Gauss-Legendre nodes/weights on [-1, 1] (library routine)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def curve(shape: int, a: float, c: float, kappa: float, t):
    """Generating curve and centreline at parameter t (latitude).

    Returns r, dr, z, dz, p, dp, q, dq (derivatives with respect to t).
    sphere/spheroid: r = a cos t, z = c sin t.
    peanut: polar radius a (1 + c cos 2 psi), psi = pi/2 - t the polar angle,
            i.e. rho(t) = a (1 - c cos 2t), r = rho cos t, z = rho sin t.
    The three geometries of Section 6.1, Example 2 (equations quasiellipsoid,
    spiral, conch), scaled by a (c and kappa unused):
    quasi-ellipsoid: r = 2a cos t, z = 3a sin t, p = a cos t, q = 0;
    spiral: r = 1.5a cos t, z = 2a sin t, p = 0.05a cos 4 pi t, q = 0.1a sin 4 pi t;
    conch: r = a cos t, z = 1.5a sin t, p = a f cos t, q = a f sin t,
           f = 0.2 + 0.1 sin 8t.
    """
    t = np.asarray(t, dtype=np.float64)
    if shape in (QUASI_ELLIPSOID, SPIRAL, CONCH):
        ct, st = np.cos(t), np.sin(t)
        if shape == QUASI_ELLIPSOID:
            r, dr, z, dz = 2 * a * ct, -2 * a * st, 3 * a * st, 3 * a * ct
            p, dp = a * ct, -a * st
            q, dq = np.zeros_like(t), np.zeros_like(t)
        elif shape == SPIRAL:
            w = 4 * np.pi
            r, dr, z, dz = 1.5 * a * ct, -1.5 * a * st, 2 * a * st, 2 * a * ct
            p, dp = 0.05 * a * np.cos(w * t), -0.05 * a * w * np.sin(w * t)
            q, dq = 0.1 * a * np.sin(w * t), 0.1 * a * w * np.cos(w * t)
        else:
            f, df = 0.2 + 0.1 * np.sin(8 * t), 0.8 * np.cos(8 * t)
            r, dr, z, dz = a * ct, -a * st, 1.5 * a * st, 1.5 * a * ct
            p, dp = a * f * ct, a * (df * ct - f * st)
            q, dq = a * f * st, a * (df * st + f * ct)
        return r, dr, z, dz, p, dp, q, dq
    if shape in (SPHERE, SPHEROID):
        r = a * np.cos(t)
        dr = -a * np.sin(t)
        z = c * np.sin(t)
        dz = c * np.cos(t)
    elif shape == PEANUT:
        rho = a * (1.0 - c * np.cos(2 * t))
        drho = 2.0 * a * c * np.sin(2 * t)
        r = rho * np.cos(t)
        dr = drho * np.cos(t) - rho * np.sin(t)
        z = rho * np.sin(t)
        dz = drho * np.sin(t) + rho * np.cos(t)
    else:
        raise ValueError(f"unknown shape {shape}")
    if kappa != 0.0:
        root = np.sqrt(1.0 - (kappa * z) ** 2)
        p = kappa * z * z / (1.0 + root)
        dp = kappa * z / root * dz
    else:
        p = np.zeros_like(t)
        dp = np.zeros_like(t)
    q = np.zeros_like(t)
    dq = np.zeros_like(t)
    return r, dr, z, dz, p, dp, q, dq


def curve_differences(shape: int, a: float, c: float, kappa: float, t, dl):
    """Cancellation-free differences between the slice at s = t + dl and the
    slice at t:  dr = r(s) - r(t), dz = z(t) - z(s), dp = p(t) - p(s),
    dq = q(t) - q(s).  Written with sin(dl/2) (product-to-sum identities) so
    that they keep full relative accuracy as dl -> 0; needed because the
    singular quadrature places nodes very close to the target.
    """
    t = np.asarray(t, dtype=np.float64)
    dl = np.asarray(dl, dtype=np.float64)
    s = t + dl
    sig = t + 0.5 * dl
    sh = np.sin(0.5 * dl)
    dcos = -2.0 * np.sin(sig) * sh                       # cos s - cos t
    dsin = -2.0 * np.cos(sig) * sh                       # sin t - sin s
    if shape == QUASI_ELLIPSOID:
        return 2 * a * dcos, 3 * a * dsin, -a * dcos, np.zeros_like(dcos)
    if shape == SPIRAL:
        w = 4 * np.pi
        # cos wt - cos ws = 2 sin(w sig) sin(w dl / 2); sin wt - sin ws = -2 cos(w sig) sin(w dl / 2)
        sw = np.sin(0.5 * w * dl)
        return (1.5 * a * dcos, 2 * a * dsin, 0.1 * a * np.sin(w * sig) * sw,
                -0.2 * a * np.cos(w * sig) * sw)
    if shape == CONCH:
        f_s = 0.2 + 0.1 * np.sin(8 * s)
        df = -0.2 * np.cos(8 * sig) * np.sin(4 * dl)      # f(t) - f(s)
        d_p = a * (df * np.cos(t) - f_s * dcos)
        d_q = a * (df * np.sin(t) + f_s * dsin)
        return a * dcos, 1.5 * a * dsin, d_p, d_q
    if shape in (SPHERE, SPHEROID):
        d_r = -2.0 * a * np.sin(sig) * sh                 # a (cos s - cos t)
        d_z = -2.0 * c * np.cos(sig) * sh                 # c (sin t - sin s)
        z_t, z_s = c * np.sin(t), c * np.sin(s)
    elif shape == PEANUT:
        rho_t = a * (1.0 - c * np.cos(2 * t))
        rho_s = a * (1.0 - c * np.cos(2 * s))
        d_rho = 2.0 * a * c * np.sin(2 * sig) * np.sin(dl)   # rho(s) - rho(t)
        d_r = d_rho * np.cos(s) + rho_t * dcos
        d_z = rho_t * dsin - d_rho * np.sin(s)
        z_t, z_s = rho_t * np.sin(t), rho_s * np.sin(s)
    else:
        raise ValueError(f"unknown shape {shape}")
    if kappa != 0.0:
        R_t = np.sqrt(1.0 - (kappa * z_t) ** 2)
        R_s = np.sqrt(1.0 - (kappa * z_s) ** 2)
        d_p = kappa * d_z * (z_t + z_s) / (R_t + R_s)
    else:
        d_p = np.zeros_like(d_r)
    d_q = np.zeros_like(d_r)
    return d_r, d_z, d_p, d_q


def rotation(theta1: float, theta2: float) -> np.ndarray:
    """R = Rz(theta1) Ry(theta2) (Section 6.2, Example 5)."""
    c1, s1 = math.cos(theta1), math.sin(theta1)
    c2, s2 = math.cos(theta2), math.sin(theta2)
    rz = np.array([[c1, -s1, 0.0], [s1, c1, 0.0], [0.0, 0.0, 1.0]])
    ry = np.array([[c2, 0.0, s2], [0.0, 1.0, 0.0], [-s2, 0.0, c2]])
    return rz @ ry


def surface_point_normal(shape, a, c, kappa, t, theta):
    """Body-frame point y and area normal N = d_theta x d_s (|N| = |J|).

    d_s = (r' cos th + p', r' sin th + q', z'), d_theta = (-r sin th, r cos th, 0)
    (Section 3.1).  t and theta broadcast together.
    """
    r, dr, z, dz, p, dp, q, dq = curve(shape, a, c, kappa, t)
    ct, st = np.cos(theta), np.sin(theta)
    y = np.stack(np.broadcast_arrays(r * ct + p, r * st + q, z + 0 * ct), axis=-1)
    ds = np.stack(np.broadcast_arrays(dr * ct + dp, dr * st + dq, dz + 0 * ct), axis=-1)
    dth = np.stack(np.broadcast_arrays(-r * st, r * ct, 0 * r * ct), axis=-1)
    n = np.cross(dth, ds)
    return y, n


@dataclass
class BodyDisc:
    """Discretisation of one body in its own frame."""
    shape: int
    a: float
    c: float
    kappa: float
    n_panels: int            # panels after refinement
    n_theta: int
    t_nodes: np.ndarray      # (n_panels*16,) GL parameters, panel-major
    omega: np.ndarray        # (n_panels*16,) scaled GL weights
    panel_edges: np.ndarray  # (n_panels+1,)
    theta: np.ndarray        # (n_theta,)
    y0: np.ndarray           # (n, 3) body-frame nodes; order panel, GL, azimuth
    n0: np.ndarray           # (n, 3) body-frame area normals d_theta x d_s
    w: np.ndarray            # (n,) smooth weight (pi/N) omega (without |J|)

    @property
    def n(self) -> int:
        return self.y0.shape[0]


def panel_edges(n_panels: int, n_ref: int = 0) -> np.ndarray:
    """Breakpoints of the generating curve's parameter interval: n_panels
    uniform panels, then the panel at each end halved n_ref times toward
    the pole (dyadic refinement, the N_ref of the notation table of
    Section 6), n_panels + 2 n_ref panels in all."""
    h = (T1 - T0) / n_panels
    uni = T0 + h * np.arange(n_panels + 1)
    if n_ref == 0:
        return uni
    if n_panels < 2:
        raise ValueError("dyadic refinement needs at least two uniform panels")
    low = T0 + h * 2.0 ** -np.arange(n_ref, 0, -1)      # T0 + h/2^n_ref, ..., T0 + h/2
    high = T1 - h * 2.0 ** -np.arange(1, n_ref + 1)     # T1 - h/2, ..., T1 - h/2^n_ref
    return np.concatenate([[T0], low, uni[1:-1], high, [T1]])


def discretize_body(shape, a, c, kappa, n_panels, n_theta, n_ref=0) -> BodyDisc:
    """Panels x 16 GL nodes in t (n_panels uniform panels, each end panel
    refined n_ref times), 2N = n_theta trapezoid nodes in theta."""
    xg, wg = gauss_legendre(GL_ORDER)
    edges = panel_edges(n_panels, n_ref)
    n_panels = len(edges) - 1
    hp = np.diff(edges)
    t_nodes = (edges[:-1, None] + 0.5 * hp[:, None] * (xg[None, :] + 1.0)).ravel()
    omega = (0.5 * hp[:, None] * wg[None, :]).ravel()
    N = n_theta // 2
    theta = np.arange(n_theta) * math.pi / N
    tt, th = np.meshgrid(t_nodes, theta, indexing="ij")
    y, nn = surface_point_normal(shape, a, c, kappa, tt, th)
    w = np.repeat(omega, n_theta) * (math.pi / N)
    return BodyDisc(shape, a, c, kappa, n_panels, n_theta, t_nodes, omega, edges,
                    theta, y.reshape(-1, 3), nn.reshape(-1, 3), w)


@dataclass
class Discretization:
    """All nodes of a scenario in world coordinates."""
    pos: np.ndarray      # (N, 3)
    aw: np.ndarray       # (N, 3) area-weighted normal n |J| (pi/N) omega
    body: np.ndarray     # (N,) body index
    problem: np.ndarray  # (N,) problem index
    offsets: np.ndarray  # (n_bodies+1,)
    bodies: list         # BodyDisc per body
    rots: list           # R per body
    centres: np.ndarray  # (n_bodies, 3)


def discretize(scenario) -> Discretization:
    b = scenario.bodies
    pos, aw, bid, pid, discs, rots = [], [], [], [], [], []
    off = [0]
    for i in range(len(b)):
        n_ref = int(b["n_ref"][i]) if "n_ref" in b.dtype.names else 0
        d = discretize_body(int(b["shape"][i]), float(b["a"][i]), float(b["c"][i]),
                            float(b["kappa"][i]), int(b["n_panels"][i]), int(b["n_theta"][i]), n_ref)
        R = rotation(float(b["theta1"][i]), float(b["theta2"][i]))
        cen = np.array([b["cx"][i], b["cy"][i], b["cz"][i]], dtype=np.float64)
        pos.append(d.y0 @ R.T + cen)
        aw.append((d.n0 @ R.T) * d.w[:, None])
        bid.append(np.full(d.n, i, dtype=np.int64))
        pid.append(np.full(d.n, int(b["problem"][i]), dtype=np.int64))
        discs.append(d)
        rots.append(R)
        off.append(off[-1] + d.n)
    cen = np.stack([b["cx"], b["cy"], b["cz"]], axis=1).astype(np.float64)
    return Discretization(np.concatenate(pos), np.concatenate(aw), np.concatenate(bid),
                          np.concatenate(pid), np.array(off, dtype=np.int64), discs, rots, cen)
