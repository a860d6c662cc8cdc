"""Oracle self-interaction block B_b = 1/2 I + D_bb of one body (Sections 3.1-3.4).

Row T (target x on panel p), column (i, l, j) (panel, GL node, azimuth):

  near panels: i in {p-1, p, p+1}, and any panel on whose rings the smooth
  rule's trapezoid in theta would not resolve the kernel (see panel_is_near)
  (Section 3.1, equations muJ / coef_ele, Section 3.4):
                 E = int_{gamma_i} P_il(s) G_j(x, s) ds,
                 G_j(x, s) = int_0^{2pi} K(x, y(s, theta)) L_j(theta) dtheta,
                 K = grad_y G^k . (d_theta x d_s)   (density mu interpolated);
  far panels     (Section 3.1, equation sx): E = K(x, y_ilj) (pi/N) omega_il.

The outer s-integral has a logarithmic singularity at s = t (self panel) and a
near singularity at the shared end of an adjacent panel.  The paper uses
generalized Gaussian quadrature tables that are not available; this oracle
uses composite Gauss-Legendre on geometrically graded subintervals (ratio 1/4,
24 levels, pieces no longer than 0.1) toward the singular point instead, which
converges to the same integrals (two such rules of different density agree to
about 1e-13 relative).
G_j is evaluated by the modal route (recurrence + FFT + convolution, Section
3.3) when chi - 1 < CHI_SPLIT and by the trapezoidal rule on the kernel itself
otherwise.
"""
from __future__ import annotations

import math

import numpy as np

from . import geometry as geo
from . import modal

CHI_SPLIT = 0.08      # below: modal route; above: direct trapezoid
L_DIRECT = 256
L_MODAL = 256
RATIO = 0.25
N_SUB = 16
H_MAX = 0.1           # longest graded subinterval (resolves the azimuthal structure of G_j)
NEAR_EXP = 40.0       # smooth rule only where the trapezoid's aliased modes are below e^-40


def lagrange_gl(nodes, s):
    """P_l(s) for the Lagrange basis on the given nodes: (len(s), len(nodes))."""
    s = np.asarray(s)[:, None]
    x = np.asarray(nodes)[None, :]
    n = len(nodes)
    out = np.ones((s.shape[0], n))
    for l in range(n):
        for m in range(n):
            if m != l:
                out[:, l] *= (s[:, 0] - nodes[m]) / (nodes[l] - nodes[m])
    return out


def graded_rule(s0, s1, levels, ratio=RATIO, n=N_SUB, hmax=H_MAX):
    """Gauss-Legendre on subintervals of [s0, s1] graded geometrically toward s0,
    each subinterval split further into pieces no longer than hmax.
    Returns offsets u = s - s0 and weights."""
    xg, wg = geo.gauss_legendre(n)
    ell = s1 - s0
    bps = [ell * ratio ** kk for kk in range(levels + 1)] + [0.0]
    S, W = [], []
    for a, b in zip(bps[:-1], bps[1:]):
        m = max(1, int(math.ceil(abs(b - a) / hmax)))
        for q in range(m):
            y0 = a + (b - a) * q / m
            y1 = a + (b - a) * (q + 1) / m
            h = 0.5 * (y1 - y0)
            S.append(0.5 * (y0 + y1) + h * xg)
            W.append(abs(h) * wg)
    return np.concatenate(S), np.concatenate(W)


def panel_is_near(disc: geo.BodyDisc, pT: int, tT: float, thT: float, i: int) -> bool:
    """Product integration for panel i (target at (tT, thT) on panel pT): the
    adjacent panels always, and any panel on which the smooth rule of
    Section 3.1 (equation sx) would fail in theta.  The kernel's azimuthal
    modes on a ring decay like e^{-|m| acosh chi}, so the trapezoidal rule on
    2N points is exact to e^{-2N acosh chi}; near a pole of a dyadically
    refined curve, panels two or more apart can still have chi - 1 = O(1)
    (the rings shrink with the panels).  Reading: the paper only names
    adjacent panels as near; this criterion keeps its smooth rule where it is
    accurate and extends product integration where it is not."""
    if abs(i - pT) <= 1:
        return True
    s = disc.t_nodes[i * geo.GL_ORDER:(i + 1) * geo.GL_ORDER]
    loc = modal.local_frame_rel(disc.shape, disc.a, disc.c, disc.kappa, np.full(s.shape, tT),
                                np.full(s.shape, thT), s - tT)
    chim1 = loc["chim1"]
    acosh = np.log1p(chim1 + np.sqrt(chim1 * (chim1 + 2.0)))
    return bool(np.any(disc.n_theta * acosh < NEAR_EXP))


def outer_rule(disc: geo.BodyDisc, pT: int, tT: float, i: int):
    """Outer nodes on near panel i for the target at tT: offsets dl = s - tT and
    weights.  Self panel: split at tT, graded toward tT down to 1e-14 of the
    sub-interval length.  Adjacent panel: graded toward the shared end."""
    e = disc.panel_edges
    if i == pT:
        out_s, out_w = [], []
        for end in (e[i], e[i + 1]):
            ell = abs(end - tT)
            levels = int(math.ceil(math.log(1e14) / math.log(1.0 / RATIO)))
            u, w = graded_rule(0.0, end - tT, levels)
            out_s.append(u)
            out_w.append(w)
        return np.concatenate(out_s), np.concatenate(out_w)
    if i < pT:
        end, far = e[i + 1], e[i]
    else:
        end, far = e[i], e[i + 1]
    d = abs(tT - end)
    levels = max(1, int(math.ceil(math.log(abs(far - end) / d) / math.log(1.0 / RATIO))) + 1)
    u, w = graded_rule(0.0, far - end, levels)
    return (end - tT) + u, w


def slice_geometry(disc: geo.BodyDisc, s):
    r, dr, z, dz, p, dp, q, dq = geo.curve(disc.shape, disc.a, disc.c, disc.kappa, s)
    return {"r": r, "dr": dr, "z": z, "dz": dz, "p": p, "dp": dp, "q": q, "dq": dq}


def gj(k, N, disc, t_t, th_t, dl):
    """G_j(x, s) for many (target, s = t_t + dl) pairs; modal route when
    chi - 1 < CHI_SPLIT, direct trapezoid otherwise."""
    loc = modal.local_frame_rel(disc.shape, disc.a, disc.c, disc.kappa, t_t, th_t, dl)
    out = np.zeros((t_t.shape[0], 2 * N), dtype=np.complex128)
    near = loc["chim1"] < CHI_SPLIT
    if np.any(near):
        out[near] = modal.gj_modal(k, N, {kk: v[near] for kk, v in loc.items()}, L=L_MODAL)
    if np.any(~near):
        far = ~near
        x, _ = geo.surface_point_normal(disc.shape, disc.a, disc.c, disc.kappa, t_t[far], th_t[far])
        sg = slice_geometry(disc, t_t[far] + dl[far])
        out[far] = modal.gj_direct(k, N, x, sg, L=L_DIRECT)
    return out


def gj_sl(k, N, disc, t_t, th_t, dl):
    """Single-layer G^S_j for many (target, s) pairs, routes as in gj."""
    loc = modal.local_frame_rel(disc.shape, disc.a, disc.c, disc.kappa, t_t, th_t, dl)
    out = np.zeros((t_t.shape[0], 2 * N), dtype=np.complex128)
    near = loc["chim1"] < CHI_SPLIT
    if np.any(near):
        out[near] = modal.gj_sl_modal(k, N, {kk: v[near] for kk, v in loc.items()}, L=L_MODAL)
    if np.any(~near):
        far = ~near
        x, _ = geo.surface_point_normal(disc.shape, disc.a, disc.c, disc.kappa, t_t[far], th_t[far])
        sg = slice_geometry(disc, t_t[far] + dl[far])
        out[far] = modal.gj_sl_direct(k, N, x, sg, L=L_DIRECT)
    return out


def self_block(disc: geo.BodyDisc, k: float, rows=None, chunk=4000, kind="dl"):
    """Rows of B = 1/2 I + D (kind "dl") or of the single-layer block S
    (kind "sl": the density times |J| is interpolated, so column (i, l, j)
    carries |J| at its node; far panels use G |J| (pi/N) omega) for one body
    in its own frame (complex128)."""
    n = disc.n
    nth = disc.n_theta
    N = nth // 2
    per_panel = geo.GL_ORDER * nth
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.zeros((rows.shape[0], n), dtype=np.complex128)
    # gather (row, panel, s, w) for near panels
    rec_row, rec_pan, rec_s, rec_w = [], [], [], []
    for ri, T in enumerate(rows):
        pT = T // per_panel
        lT = (T // nth) % geo.GL_ORDER
        tT = disc.t_nodes[pT * geo.GL_ORDER + lT]
        thT = disc.theta[T % nth]
        for i in range(disc.n_panels):
            if panel_is_near(disc, pT, tT, thT, i):
                s, w = outer_rule(disc, pT, tT, i)
                rec_row.append(np.full(s.shape, ri))
                rec_pan.append(np.full(s.shape, i))
                rec_s.append(s)
                rec_w.append(w)
            else:
                cols = slice(i * per_panel, (i + 1) * per_panel)
                if kind == "sl":
                    # |J| of the column is applied to the whole row below
                    out[ri, cols] = modal.sl_kernel(k, disc.y0[T][None, :], disc.y0[cols]) * disc.w[cols]
                else:
                    out[ri, cols] = modal.dl_kernel_area(
                        k, disc.y0[T][None, :], disc.y0[cols], disc.n0[cols]) * disc.w[cols]
    rr = np.concatenate(rec_row)
    pp = np.concatenate(rec_pan)
    ss = np.concatenate(rec_s)      # offsets dl = s - t_T
    ww = np.concatenate(rec_w)
    t_row = disc.t_nodes[(rows // per_panel) * geo.GL_ORDER + (rows // nth) % geo.GL_ORDER]
    th_row = disc.theta[rows % nth]
    for c0 in range(0, rr.shape[0], chunk):
        sl = slice(c0, c0 + chunk)
        tt = t_row[rr[sl]]
        G = (gj_sl if kind == "sl" else gj)(k, N, disc, tt, th_row[rr[sl]], ss[sl])   # (P, 2N)
        s_abs = tt + ss[sl]
        for i in np.unique(pp[sl]):
            m = pp[sl] == i
            gl_nodes = disc.t_nodes[i * geo.GL_ORDER:(i + 1) * geo.GL_ORDER]
            Pl = lagrange_gl(gl_nodes, s_abs[m]) * ww[sl][m][:, None]   # (P_i, 16)
            contrib = Pl[:, :, None] * G[m][:, None, :]                 # (P_i, 16, 2N)
            rows_i = rr[sl][m]
            cols = slice(i * per_panel, (i + 1) * per_panel)
            blk = np.zeros((rows.shape[0], per_panel), dtype=np.complex128)
            np.add.at(blk, rows_i, contrib.reshape(contrib.shape[0], -1))
            out[:, cols] += blk
    if kind == "sl":
        out *= np.linalg.norm(disc.n0, axis=1)[None, :]       # |J| of the column node
        return out
    out[np.arange(rows.shape[0]), rows] += 0.5
    return out


def self_block_cf(disc: geo.BodyDisc, k: float, eta: float, rows=None):
    """Rows of the combined-field block 1/2 I + D - i eta S (the remark on
    combined fields in Section 2)."""
    return self_block(disc, k, rows) - 1j * eta * self_block(disc, k, rows, kind="sl")
