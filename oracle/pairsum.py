"""Oracle inter-body double-layer pair sum (Section 4, the display after the
equation labelled multi2part): for target x_i and every source node y_j on a
different body of the same problem,

  w_i = sum_j (ik/|x-y| - 1/|x-y|^2) e^{ik|x-y|}/(4 pi |x-y|) n(y).(y - x) mu_j |J| (pi/N) omega,

i.e. the direct double loop (no compression).  ``aw`` holds n |J| (pi/N) omega.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def pair_sum(disc, k_per_problem, mu, targets=None, chunk=256, eta=None, single=False):
    """mu: (N,) or (N, nrhs) complex.  Returns w at the requested targets.
    single: the single-layer kernel G(x, y_j) |J_j| w_j alone (the first-kind
    equation of Section 2).
    With eta, the combined-field kernel: double layer - i eta single layer,
    the single layer as G(x, y_j) |J_j| w_j (|J| w = |aw|)."""
    mu = np.asarray(mu, dtype=np.complex128)
    squeeze = mu.ndim == 1
    if squeeze:
        mu = mu[:, None]
    targets = np.arange(disc.pos.shape[0]) if targets is None else np.asarray(targets)
    out = np.zeros((targets.shape[0], mu.shape[1]), dtype=np.complex128)
    for c0 in range(0, targets.shape[0], chunk):
        ti = targets[c0:c0 + chunk]
        probs = disc.problem[ti]
        for p in np.unique(probs):
            k = float(k_per_problem[p])
            sel = np.nonzero(probs == p)[0]
            tsel = ti[sel]
            src = np.nonzero(disc.problem == p)[0]
            d = disc.pos[src][None, :, :] - disc.pos[tsel][:, None, :]      # y - x
            rho = np.sqrt(np.sum(d * d, axis=-1))
            same = disc.body[tsel][:, None] == disc.body[src][None, :]
            rho_safe = np.where(same, 1.0, rho)
            if single:
                kern = np.exp(1j * k * rho_safe) / (FOUR_PI * rho_safe) \
                    * np.linalg.norm(disc.aw[src], axis=1)[None, :]
            else:
                kern = (1j * k / rho_safe - 1.0 / rho_safe ** 2) * np.exp(1j * k * rho_safe) \
                    / (FOUR_PI * rho_safe) * np.sum(disc.aw[src][None, :, :] * d, axis=-1)
            if eta is not None and not single:
                w = np.linalg.norm(disc.aw[src], axis=1)[None, :]
                kern = kern - 1j * eta * np.exp(1j * k * rho_safe) / (FOUR_PI * rho_safe) * w
            kern = np.where(same, 0.0, kern)
            out[c0 + sel] = kern @ mu[src]
    return out[:, 0] if squeeze else out


def pair_sum_bruteforce(disc, k_per_problem, mu):
    """Pure-Python double loop (tiny inputs only)."""
    n = disc.pos.shape[0]
    out = np.zeros(n, dtype=np.complex128)
    for i in range(n):
        acc = 0j
        for j in range(n):
            if disc.body[i] == disc.body[j] or disc.problem[i] != disc.problem[j]:
                continue
            k = float(k_per_problem[disc.problem[i]])
            dx = disc.pos[j] - disc.pos[i]
            rho = math.sqrt(float(dx @ dx))
            g = complex(math.cos(k * rho), math.sin(k * rho)) / (FOUR_PI * rho)
            acc += (1j * k / rho - 1.0 / rho ** 2) * g * float(disc.aw[j] @ dx) * mu[j]
        out[i] = acc
    return out
