"""Block reuse on regular arrays of identical bodies (test infrastructure).

Section 4, the paragraph on identical scatterers on a regular P x Q x R array
with uniform spacing: the interaction block between bodies t' and t depends
only on the displacement d = c_t' - c_t of their centres, so the
N_geo (N_geo - 1) off-diagonal blocks reduce to (2P-1)(2Q-1)(2R-1) - 1
distinct ones; each is computed once by quadrature and reused for every pair
with that displacement (the block reuse ratio of Table 7).

Here:
* `distinct_displacements` / `reuse_ratio` count by enumerating every
  ordered pair of distinct sites (brute force, not the closed form);
* `displacement_block` is one representative block D_d by the smooth rule of
  Section 3.1 (equation sx), the pair-sum kernel between the nodes of a body
  displaced by d and those of the reference body;
* `lattice_apply` evaluates the inter-body sum of Section 4 with every
  off-diagonal block taken from the table by its displacement.

Only tests may import this module.  Reading (the paper does not fix it): the
array axes are the coordinate axes, spacing may differ per axis, and bodies
may be listed in any order (sites are recovered from the centres).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import modal

FOUR_PI = 4.0 * np.pi


def lattice_sites(centres, rtol=1e-12):
    """Sites (n_bodies, 3) integer indices, dims (P, Q, R) and spacing of
    centres on a full regular array aligned with the axes; ValueError
    otherwise."""
    c = np.asarray(centres, dtype=np.float64)
    scale = max(1.0, float(np.abs(c).max()))
    dims, spacing, idx = [], [], []
    for ax in range(3):
        u = np.unique(c[:, ax])
        merged = [u[0]]
        for v in u[1:]:
            if v - merged[-1] > rtol * scale * 1e3:
                merged.append(v)
        u = np.array(merged)
        n = len(u)
        h = (u[-1] - u[0]) / (n - 1) if n > 1 else 0.0
        if n > 1 and np.abs(u - (u[0] + h * np.arange(n))).max() > rtol * scale * 1e3:
            raise ValueError("centres are not uniformly spaced")
        i = np.rint((c[:, ax] - u[0]) / h).astype(np.int64) if n > 1 else np.zeros(len(c), np.int64)
        dims.append(n)
        spacing.append(h)
        idx.append(i)
    sites = np.stack(idx, axis=1)
    P, Q, R = dims
    if P * Q * R != len(c) or len({tuple(s) for s in sites}) != len(c):
        raise ValueError("centres do not fill a regular array")
    return sites, (P, Q, R), np.array(spacing)


def distinct_displacements(P, Q, R):
    """Displacements d = site' - site over all ordered pairs of distinct sites."""
    sites = list(itertools.product(range(P), range(Q), range(R)))
    seen = set()
    for a in sites:
        for b in sites:
            if a != b:
                seen.add((a[0] - b[0], a[1] - b[1], a[2] - b[2]))
    return sorted(seen)


def reuse_ratio(P, Q, R):
    """1 - (distinct off-diagonal blocks) / (all off-diagonal blocks)."""
    n = P * Q * R
    return 1.0 - len(distinct_displacements(P, Q, R)) / (n * (n - 1))


def displacement_block(disc, k, d_vec, ref=0, eta=None, single=False):
    """D_d[i, j]: the pair-sum kernel from source node j of body `ref` to
    target node i of the same body translated by d_vec (smooth rule, the
    weights in aw)."""
    o0, o1 = disc.offsets[ref], disc.offsets[ref + 1]
    y = disc.pos[o0:o1]
    aw = disc.aw[o0:o1]
    x = y + np.asarray(d_vec, dtype=np.float64)[None, :]
    if single:
        return modal.sl_kernel(k, x[:, None, :], y[None, :, :]) * np.linalg.norm(aw, axis=1)[None, :]
    D = modal.dl_kernel_area(k, x[:, None, :], y[None, :, :], aw[None, :, :])
    if eta is not None:
        D = D - 1j * eta * modal.sl_kernel(k, x[:, None, :], y[None, :, :]) \
            * np.linalg.norm(aw, axis=1)[None, :]
    return D


def block_table(disc, k, dims, spacing, eta=None, single=False):
    """{d: D_d} for every distinct displacement of the array."""
    return {d: displacement_block(disc, k, np.array(d) * spacing, eta=eta, single=single)
            for d in distinct_displacements(*dims)}


def lattice_apply(disc, k, mu, eta=None, single=False):
    """w_t' = sum_{t != t'} D_{c_t' - c_t} mu_t with the blocks from the table.
    mu (N,) or (N, nrhs)."""
    mu = np.asarray(mu, dtype=np.complex128)
    squeeze = mu.ndim == 1
    if squeeze:
        mu = mu[:, None]
    sites, dims, spacing = lattice_sites(disc.centres)
    table = block_table(disc, k, dims, spacing, eta=eta, single=single)
    off = disc.offsets
    out = np.zeros_like(mu)
    nb = len(off) - 1
    for tp in range(nb):
        for t in range(nb):
            if t == tp:
                continue
            d = tuple(int(v) for v in sites[tp] - sites[t])
            out[off[tp]:off[tp + 1]] += table[d] @ mu[off[t]:off[t + 1]]
    return out[:, 0] if squeeze else out
