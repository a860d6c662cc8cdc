"""Seeded synthetic scenario generators (inputs only).

This module draws the random inputs of every workload -- which shape each body
has, its centreline curvature, its two rotation angles, its centre, its
discretisation, the wavenumber of each problem and the incident directions --
and nothing else.  It holds none of the method's arithmetic: no rotation
matrices, no surface nodes, no kernels.  Both the HIP library (through the
Python binding) and the CPU oracle consume the descriptors it returns.

Every generator uses numpy's PCG64 with an explicit seed.

Body descriptor fields (one row of ``BODY_DTYPE``):

``shape``      0 = sphere, 1 = spheroid, 2 = peanut, 3 = quasi-ellipsoid,
               4 = spiral, 5 = conch (the last three: Section 6.1, Example 2)
``a``, ``c``   sphere: radius ``a`` (``c`` = ``a``); spheroid: radial semi-axis
               ``a`` and axial semi-axis ``c``; peanut: polar radius
               ``a (1 + c cos 2 psi)`` with ``psi`` the polar angle;
               shapes 3-5: scale ``a`` (``c`` unused)
``kappa``      curvature of the circular-arc centreline (0 = straight axis;
               shapes 3-5: 0)
``n_panels``   uniform Gauss-Legendre panels along the generating curve (16
               nodes each)
``n_ref``      dyadic refinements of the panel at each pole (adds 2 n_ref panels)
``n_theta``    azimuthal trapezoidal nodes (even, 2N)
``theta1``, ``theta2``  rotation angles of R = Rz(theta1) Ry(theta2)
``cx, cy, cz`` body centre
``problem``    index of the independent scattering problem the body belongs to

Paper context: random rigid motions of identical bodies (Section 6.2, Example
5); plane-wave direction angles theta = pi/3, phi = 2 pi/3 (Section 6, the
plane-wave parameters equation).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

SPHERE, SPHEROID, PEANUT = 0, 1, 2
QUASI_ELLIPSOID, SPIRAL, CONCH = 3, 4, 5
GL_ORDER = 16

BODY_DTYPE = np.dtype([
    ("shape", np.int32), ("a", np.float64), ("c", np.float64),
    ("kappa", np.float64), ("n_panels", np.int32), ("n_theta", np.int32),
    ("theta1", np.float64), ("theta2", np.float64),
    ("cx", np.float64), ("cy", np.float64), ("cz", np.float64),
    ("problem", np.int32), ("n_ref", np.int32),
])


@dataclass
class Scenario:
    name: str
    bodies: np.ndarray                     # BODY_DTYPE records
    k: np.ndarray                          # wavenumber per problem
    dirs: np.ndarray                       # (nrhs, 3) incident directions (per problem: same set)
    tol: float = 1e-8
    solver: str = "gmres"                  # "gmres" or "dense"
    notes: dict = field(default_factory=dict)

    @property
    def n_problems(self) -> int:
        return int(self.k.shape[0])

    def nodes_per_body(self) -> np.ndarray:
        panels = self.bodies["n_panels"].astype(np.int64) + 2 * self.bodies["n_ref"].astype(np.int64)
        return panels * GL_ORDER * self.bodies["n_theta"].astype(np.int64)

    def n_unknowns(self) -> int:
        return int(self.nodes_per_body().sum())

    def pairs_per_apply(self) -> int:
        """Inter-body (target, source) node pairs of one operator apply, per RHS."""
        n = self.nodes_per_body()
        tot = 0
        for p in range(self.n_problems):
            m = self.bodies["problem"] == p
            s = int(n[m].sum())
            tot += s * s - int((n[m] ** 2).sum())
        return tot


def paper_direction() -> np.ndarray:
    """d = (cos t sin f, sin t sin f, cos f) with t = pi/3, f = 2 pi/3."""
    t, f = math.pi / 3, 2 * math.pi / 3
    return np.array([[math.cos(t) * math.sin(f), math.sin(t) * math.sin(f), math.cos(f)]])


def bounding_radius(shape: int, a: float, c: float, kappa: float) -> float:
    """Generous radius of a ball about the body centre that contains the body."""
    if shape == SPHERE:
        zmax, rmax = a, a
    elif shape == SPHEROID:
        zmax, rmax = c, a
    else:
        zmax, rmax = a * (1 + c), a * (1 + c)
    off = kappa * zmax * zmax  # generous bound on the centreline offset
    return math.hypot(rmax + off, zmax)


def make_bodies(n: int) -> np.ndarray:
    return np.zeros(n, dtype=BODY_DTYPE)


def _fill(b, shape, a, c, kappa, n_panels, n_theta, t1, t2, centre, problem=0):
    b["shape"], b["a"], b["c"], b["kappa"] = shape, a, c, kappa
    b["n_panels"], b["n_theta"] = n_panels, n_theta
    b["theta1"], b["theta2"] = t1, t2
    b["cx"], b["cy"], b["cz"] = centre
    b["problem"] = problem


def _rejection_centres(rng, n, radii, half_side, gap, max_tries=2_000_000):
    """Centres uniform in [-half_side, half_side]^3 with |ci-cj| >= Ri+Rj+gap."""
    cs = np.zeros((n, 3))
    placed = 0
    tries = 0
    while placed < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("rejection sampling failed; box too small")
        p = rng.uniform(-half_side + radii[placed], half_side - radii[placed], 3)
        if placed:
            d = np.linalg.norm(cs[:placed] - p, axis=1)
            if np.any(d < radii[:placed] + radii[placed] + gap):
                continue
        cs[placed] = p
        placed += 1
    return cs


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def two_spheres(n_panels=1, n_theta=32, k=2.0) -> Scenario:
    """2 sound-soft spheres of radius 0.5 at (+-1, 0, 0); 16 GL x 32 azimuthal
    nodes each; k = 2; d = (0, 0, 1); dense LU."""
    b = make_bodies(2)
    for i, x in enumerate((-1.0, 1.0)):
        _fill(b[i], SPHERE, 0.5, 0.5, 0.0, n_panels, n_theta, 0.0, 0.0, (x, 0.0, 0.0))
    return Scenario("two_spheres", b, np.array([k]), np.array([[0.0, 0.0, 1.0]]),
                    tol=1e-12, solver="dense")


def single_sphere(a=0.5, n_panels=1, n_theta=32, k=2.0) -> Scenario:
    b = make_bodies(1)
    _fill(b[0], SPHERE, a, a, 0.0, n_panels, n_theta, 0.0, 0.0, (0.0, 0.0, 0.0))
    return Scenario("single_sphere", b, np.array([k]), np.array([[0.0, 0.0, 1.0]]),
                    tol=1e-12, solver="dense")


def lattice27(seed=0, n_panels=2, n_theta=64, k=5.0) -> Scenario:
    """27 bent prolate spheroids (0.5, 0.5, 1.0) on a 3x3x3 lattice of spacing 3,
    curvature ~U[0, 0.3], rotation angles ~U[0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = make_bodies(27)
    i = 0
    for x in (-3.0, 0.0, 3.0):
        for y in (-3.0, 0.0, 3.0):
            for z in (-3.0, 0.0, 3.0):
                kap = rng.uniform(0.0, 0.3)
                t1, t2 = rng.uniform(0.0, 2 * math.pi, 2)
                _fill(b[i], SPHEROID, 0.5, 1.0, kap, n_panels, n_theta, t1, t2, (x, y, z))
                i += 1
    return Scenario("lattice27", b, np.array([k]), paper_direction(), tol=1e-8)


def random_mixed(n_bodies=1000, seed=0, side=40.0, k=4.0) -> Scenario:
    """n_bodies of three shapes (sphere r=0.5, spheroid (0.5,0.5,1), peanut
    0.5(1+0.3 cos 2psi)), curvature ~U[0,0.3], random rotations, 16-32 GL x
    16-32 azimuthal nodes, rejection-sampled centres in a cube of given side
    with gaps of at least half a wavelength."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = make_bodies(n_bodies)
    shapes = rng.integers(0, 3, n_bodies)
    kap = rng.uniform(0.0, 0.3, n_bodies)
    t12 = rng.uniform(0.0, 2 * math.pi, (n_bodies, 2))
    npan = rng.integers(1, 3, n_bodies)
    nth = 2 * rng.integers(8, 17, n_bodies)
    params = {SPHERE: (0.5, 0.5), SPHEROID: (0.5, 1.0), PEANUT: (0.5, 0.3)}
    radii = np.array([bounding_radius(int(s), *params[int(s)], kap[i])
                      for i, s in enumerate(shapes)])
    cs = _rejection_centres(rng, n_bodies, radii, side / 2, math.pi / k)
    for i in range(n_bodies):
        s = int(shapes[i])
        _fill(b[i], s, *params[s], kap[i], int(npan[i]), int(nth[i]),
              t12[i, 0], t12[i, 1], cs[i])
    return Scenario("random_mixed", b, np.array([k]), paper_direction(), tol=1e-6)


def lattice_like_random(n_bodies=200, seed=0, side=20.0, k=6.0, nrhs=64,
                        n_panels=2, n_theta=64) -> Scenario:
    """n_bodies bent spheroids (the 27-body lattice's shape distribution) at
    rejection-sampled centres in a cube, with nrhs directions uniform on S^2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = make_bodies(n_bodies)
    kap = rng.uniform(0.0, 0.3, n_bodies)
    t12 = rng.uniform(0.0, 2 * math.pi, (n_bodies, 2))
    radii = np.array([bounding_radius(SPHEROID, 0.5, 1.0, x) for x in kap])
    cs = _rejection_centres(rng, n_bodies, radii, side / 2, math.pi / k)
    for i in range(n_bodies):
        _fill(b[i], SPHEROID, 0.5, 1.0, kap[i], n_panels, n_theta, t12[i, 0], t12[i, 1], cs[i])
    u = rng.uniform(-1.0, 1.0, nrhs)
    ph = rng.uniform(0.0, 2 * math.pi, nrhs)
    s = np.sqrt(1 - u * u)
    dirs = np.stack([s * np.cos(ph), s * np.sin(ph), u], axis=1)
    return Scenario("multi_rhs", b, np.array([k]), dirs, tol=1e-6)


def uneven_batch(n_problems=32, seed=0, max_bodies=100) -> Scenario:
    """Independent problems: each has 1..max_bodies bent spheroids, its own
    k ~ U[1, 10], 16-32 GL x 16-64 azimuthal nodes per body, centres in a cube
    with gaps of at least half a wavelength: side 2 R + (n v)^(1/3), where the
    volume per body v makes the spheres of diameter d = 2 R + pi/k fill a
    quarter of it (v = (pi/6) d^3 / 0.25; R the largest bounding radius), one
    random direction per problem (all problems share the direction array of
    the first; per-problem directions are listed in notes['dirs'])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = []
    ks = rng.uniform(1.0, 10.0, n_problems)
    dirs = []
    for p in range(n_problems):
        nb = int(rng.integers(1, max_bodies + 1))
        kap = rng.uniform(0.0, 0.3, nb)
        t12 = rng.uniform(0.0, 2 * math.pi, (nb, 2))
        npan = rng.integers(1, 3, nb)
        nth = 2 * rng.integers(8, 33, nb)
        radii = np.array([bounding_radius(SPHEROID, 0.5, 1.0, x) for x in kap])
        rmax = float(radii.max())
        dex = 2 * rmax + math.pi / ks[p]
        side = 2 * rmax + (nb * (math.pi / 6.0) * dex ** 3 / 0.25) ** (1.0 / 3.0)
        cs = _rejection_centres(rng, nb, radii, side / 2, math.pi / ks[p])
        bb = make_bodies(nb)
        for i in range(nb):
            _fill(bb[i], SPHEROID, 0.5, 1.0, kap[i], int(npan[i]), int(nth[i]),
                  t12[i, 0], t12[i, 1], cs[i], problem=p)
        rows.append(bb)
        u = rng.uniform(-1.0, 1.0)
        ph = rng.uniform(0.0, 2 * math.pi)
        s = math.sqrt(1 - u * u)
        dirs.append([s * math.cos(ph), s * math.sin(ph), u])
    b = np.concatenate(rows)
    return Scenario("uneven_batch", b, ks, np.array(dirs[:1]), tol=1e-6,
                    notes={"dirs": np.array(dirs)})


def tiny(n_bodies=2, n_panels=1, n_theta=8, k=2.0, seed=0, shapes=(SPHEROID,),
         spacing=3.0) -> Scenario:
    """A handful of small bent bodies on a line (for brute-force checks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = make_bodies(n_bodies)
    params = {SPHERE: (0.5, 0.5), SPHEROID: (0.5, 1.0), PEANUT: (0.5, 0.3)}
    for i in range(n_bodies):
        s = shapes[i % len(shapes)]
        t1, t2 = rng.uniform(0.0, 2 * math.pi, 2)
        _fill(b[i], s, *params[s], rng.uniform(0, 0.3), n_panels, n_theta, t1, t2,
              (spacing * i, 0.3 * i, -0.2 * i))
    return Scenario("tiny", b, np.array([k]), paper_direction(), tol=1e-10)


def identical_array(dims=(2, 2, 3), spacing=(3.0, 2.5, 3.5), shape=SPHEROID, a=0.5, c=1.0,
                    kappa=0.2, n_panels=1, n_theta=8, angles=(0.4, 0.9), k=2.0, seed=0,
                    shuffle=True) -> Scenario:
    """Identical bodies (same shape, curvature, orientation and
    discretisation) on a regular P x Q x R array with the given spacing per
    axis, listed in a seeded random order when `shuffle` is set."""
    P, Q, R = dims
    n = P * Q * R
    b = make_bodies(n)
    order = np.arange(n)
    if shuffle:
        order = np.random.Generator(np.random.PCG64(seed)).permutation(n)
    for slot, site in enumerate(order):
        i, rem = divmod(int(site), Q * R)
        j, l = divmod(rem, R)
        _fill(b[slot], shape, a, c, kappa, n_panels, n_theta, angles[0], angles[1],
              (spacing[0] * i, spacing[1] * j, spacing[2] * l))
    return Scenario("identical_array", b, np.array([k]), paper_direction(), tol=1e-10)


def cubic_array(P=10, n_panels=1, n_theta=6, k=2.0, spacing=3.0) -> Scenario:
    """Regular cubic array of P^3 identical bent spheroids (0.5, 0.5, 1.0),
    kappa = 0.2, one orientation, spacing 3 (gap >= 1): the block-reuse
    configuration of Example 4 (1000 bodies, 16 x 6 = 96 nodes per body),
    with bodies of the library's shape family (the quasi-ellipsoid of the
    example replaced by a bent spheroid)."""
    return identical_array((P, P, P), (spacing,) * 3, n_panels=n_panels, n_theta=n_theta, k=k,
                           shuffle=False)


WORKLOADS = {
    "two_spheres": two_spheres,
    "lattice27": lattice27,
    "random_mixed": random_mixed,
    "multi_rhs": lattice_like_random,
    "uneven_batch": uneven_batch,
}
