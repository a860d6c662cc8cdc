"""Oracle solver pieces (Sections 4 and 6).

* right-hand side -u_inc = -exp(i k d.x) (Section 2, plane wave; Section 6
  equation plane wave parameters);
* the multi-body system (1/2 I + D) mu = -u_inc in block form (Section 4,
  equation linearsys): diagonal blocks are the self blocks (identical up to
  rigid motion, so computed in the body frame), off-diagonal blocks are the
  smooth inter-body kernel;
* dense LU (numpy / LAPACK) and right-preconditioned restarted GMRES with the
  block-diagonal preconditioner built from the self blocks (Section 6, the
  paragraph on the hybrid solver);
* the combined-field variant 1/2 I + D - i eta S (eta given): single-layer
  self blocks with the density times |J| interpolated, G |J| w between bodies;
* the first-kind single-layer equation S mu = -u_inc (Section 2, equation
  single-layer-bie; `single`), the same single-layer pieces alone, far field
  (1/4 pi) sum_j e^{-i k xhat.y_j} mu_j |J_j| w_j (Section 6);
* far field of the double-layer density:
  u_inf(xhat) = (1/4 pi) sum_j (-i k xhat.n_j) e^{-i k xhat.y_j} mu_j |J_j| w_j
  (Section 6 defines the single-layer form; the double-layer form follows from
  the normal derivative of the same asymptotic expansion).
"""
from __future__ import annotations

import math

import numpy as np

from . import pairsum
from . import selfblock

FOUR_PI = 4.0 * math.pi


def rhs_planewave(disc, k_per_problem, dirs):
    """b = -exp(i k d.x); dirs (nrhs, 3).  Returns (N, nrhs)."""
    k = np.asarray(k_per_problem)[disc.problem]
    return -np.exp(1j * k[:, None] * (disc.pos @ np.asarray(dirs).T))


def self_blocks(disc, k_per_problem, body_ids=None, eta=None, single=False):
    """Self blocks 1/2 I + D (eta None), 1/2 I + D - i eta S, or S (single)."""
    body_ids = range(len(disc.bodies)) if body_ids is None else body_ids
    out = {}
    for b in body_ids:
        p = disc.problem[disc.offsets[b]]
        kp = float(k_per_problem[p])
        if single:
            out[b] = selfblock.self_block(disc.bodies[b], kp, kind="sl")
        elif eta is None:
            out[b] = selfblock.self_block(disc.bodies[b], kp)
        else:
            out[b] = selfblock.self_block_cf(disc.bodies[b], kp, eta)
    return out


def dense_matrix(disc, k_per_problem, blocks):
    """Full (1/2 I + D) as a dense matrix (small problems only)."""
    n = disc.pos.shape[0]
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        A[:, j] = pairsum.pair_sum(disc, k_per_problem, e)
    for b, B in blocks.items():
        s = slice(disc.offsets[b], disc.offsets[b + 1])
        A[s, s] = B
    return A


def dense_matrix_fast(disc, k_per_problem, blocks, eta=None, single=False):
    """Same matrix, off-diagonal entries written directly from the kernel
    (combined field with eta, single layer alone with single)."""
    n = disc.pos.shape[0]
    k = np.asarray(k_per_problem)[disc.problem]
    d = disc.pos[None, :, :] - disc.pos[:, None, :]
    rho = np.sqrt(np.sum(d * d, axis=-1))
    same = (disc.body[:, None] == disc.body[None, :]) | (disc.problem[:, None] != disc.problem[None, :])
    rs = np.where(same, 1.0, rho)
    kk = k[:, None]
    if single:
        A = np.exp(1j * kk * rs) / (FOUR_PI * rs) * np.linalg.norm(disc.aw, axis=1)[None, :]
    else:
        A = (1j * kk / rs - 1.0 / rs ** 2) * np.exp(1j * kk * rs) / (FOUR_PI * rs) \
            * np.sum(disc.aw[None, :, :] * d, axis=-1)
    if eta is not None and not single:
        A = A - 1j * eta * np.exp(1j * kk * rs) / (FOUR_PI * rs) * np.linalg.norm(disc.aw, axis=1)[None, :]
    A = np.where(same, 0.0, A)
    for b, B in blocks.items():
        s = slice(disc.offsets[b], disc.offsets[b + 1])
        A[s, s] = B
    return A


def apply_operator(disc, k_per_problem, blocks, mu, eta=None, single=False):
    """(1/2 I + D) mu (or the combined field, or S), matrix-free between bodies."""
    out = pairsum.pair_sum(disc, k_per_problem, mu, eta=eta, single=single)
    for b, B in blocks.items():
        s = slice(disc.offsets[b], disc.offsets[b + 1])
        out[s] += B @ mu[s]
    return out


def gmres(apply_a, apply_minv, b, tol=1e-10, restart=100, maxit=1000):
    """Right-preconditioned restarted GMRES (x0 = 0), classical Gram-Schmidt
    with one reorthogonalisation, Givens rotations; stops on the true relative
    residual ||b - A x|| / ||b|| <= tol.  Returns x, iterations, history."""
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    hist = []
    its = 0
    r = b.copy()
    while its < maxit:
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
        V = np.zeros((restart + 1, n), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(restart):
            w = apply_a(apply_minv(V[j]))
            h = V[: j + 1].conj() @ w
            w = w - h @ V[: j + 1]
            h2 = V[: j + 1].conj() @ w
            w = w - h2 @ V[: j + 1]
            h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0:
                V[j + 1] = w / hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(abs(H[j, j]), abs(H[j + 1, j]))
            cs[j] = abs(H[j, j]) / den if den > 0 else 1.0
            sn[j] = (H[j, j] / abs(H[j, j]) * np.conj(H[j + 1, j]) / den) if abs(H[j, j]) > 0 else 1.0
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol * 0.5 or its >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + apply_minv(y @ V[:j_end])
        r = b - apply_a(x)
    return x, its, hist


def solve(disc, k_per_problem, blocks, b, method="gmres", tol=1e-10, restart=100, maxit=1000,
          eta=None, single=False):
    """Solve (1/2 I + D) mu = b (combined field with eta, S mu = b with
    single; blocks to match); b is (N,) complex."""
    if method == "dense":
        A = dense_matrix_fast(disc, k_per_problem, blocks, eta=eta, single=single)
        return np.linalg.solve(A, b), 0, []
    inv = {bb: np.linalg.inv(B) for bb, B in blocks.items()}

    def minv(v):
        out = np.empty_like(v)
        for bb, Bi in inv.items():
            s = slice(disc.offsets[bb], disc.offsets[bb + 1])
            out[s] = Bi @ v[s]
        return out

    return gmres(lambda v: apply_operator(disc, k_per_problem, blocks, v, eta=eta, single=single), minv, b,
                 tol=tol, restart=restart, maxit=maxit)


def far_field(disc, k_per_problem, mu, xhat, eta=None, single=False, problem=0):
    """u_inf of the bodies of `problem` at unit directions xhat (ndir, 3);
    mu (N,) -> (ndir,).  With eta the combined field adds
    - i eta (1/4 pi) sum_j e^{-i k xhat.y_j} mu_j |J_j| w_j; single: that
    single-layer term alone with coefficient 1."""
    k = float(np.asarray(k_per_problem)[problem])
    sel = np.nonzero(disc.problem == problem)[0]
    pos, aw, mu = disc.pos[sel], disc.aw[sel], np.asarray(mu)[sel]
    ph = np.exp(-1j * k * (xhat @ pos.T))                 # (ndir, n)
    if single:
        return (ph * np.linalg.norm(aw, axis=1)[None, :]) @ mu / FOUR_PI
    nd = xhat @ aw.T                                       # xhat . n |J| w
    f = (-1j * k) * nd
    if eta is not None:
        f = f - 1j * eta * np.linalg.norm(aw, axis=1)[None, :]
    return (ph * f) @ mu / FOUR_PI


def near_field(disc, k_per_problem, mu, points, problem=0, chunk=64, eta=None, single=False):
    """Double-layer potential u(x) = sum_j dG/dn_y(x, y_j) mu_j |J_j| w_j of the
    bodies of `problem` at points (M, 3) away from every surface: the smooth
    product rule of Section 3.1 (equation sx) applied to the representation
    of Section 4 (equation multi-double).  mu (N,) or (N, nrhs)."""
    mu = np.asarray(mu, dtype=np.complex128)
    squeeze = mu.ndim == 1
    if squeeze:
        mu = mu[:, None]
    k = float(np.asarray(k_per_problem)[problem])
    src = np.nonzero(disc.problem == problem)[0]
    pts = np.asarray(points, dtype=np.float64)
    out = np.zeros((pts.shape[0], mu.shape[1]), dtype=np.complex128)
    for c0 in range(0, pts.shape[0], chunk):
        x = pts[c0:c0 + chunk]
        d = disc.pos[src][None, :, :] - x[:, None, :]                 # y - x
        rho = np.sqrt(np.sum(d * d, axis=-1))
        if single:
            kern = np.exp(1j * k * rho) / (FOUR_PI * rho) * np.linalg.norm(disc.aw[src], axis=1)[None, :]
        else:
            kern = (1j * k / rho - 1.0 / rho ** 2) * np.exp(1j * k * rho) / (FOUR_PI * rho) \
                * np.sum(disc.aw[src][None, :, :] * d, axis=-1)
        if eta is not None and not single:
            kern = kern - 1j * eta * np.exp(1j * k * rho) / (FOUR_PI * rho) \
                * np.linalg.norm(disc.aw[src], axis=1)[None, :]
        out[c0:c0 + chunk] = kern @ mu[src]
    return out[:, 0] if squeeze else out


def point_source_field(k, sources, x):
    """sum_s e^{i k |x - z_s|} / (4 pi |x - z_s|): a radiating solution outside
    the bodies when every z_s lies inside one (the artificial solutions of the
    numerical section).  sources (S, 3), x (M, 3) -> (M,)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape[0], dtype=np.complex128)
    for z in np.atleast_2d(sources):
        r = np.linalg.norm(x - z, axis=1)
        out += np.exp(1j * k * r) / (FOUR_PI * r)
    return out


def point_source_far_field(k, sources, xhat):
    """Far-field pattern of point_source_field with u = e^{ik|x|}/|x| u_inf:
    sum_s e^{-i k xhat.z_s} / (4 pi)."""
    return np.exp(-1j * k * (np.asarray(xhat) @ np.atleast_2d(sources).T)).sum(axis=1) / FOUR_PI
