"""Oracle modal Green's functions (Section 3.3) and the azimuthal integral
G_j(x, s) = int_0^{2 pi} K(x, y(s, theta)) L_j(theta) d theta of the
double-layer kernel (Sections 3.1-3.2).

Local geometry (Section 3.2, equations rho2 and rho-standard): for target x
and source slice s, a = x_t - p, b = y_t - q, c = z_t - z,
rt = sqrt(a^2 + b^2), alpha = arg(a + i b), phi = theta - alpha and
rho^2 = rt^2 + r^2 + c^2 - 2 r rt cos phi.  With
chi = (rt^2 + r^2 + c^2) / (2 r rt), rho = sqrt(2 r rt) sqrt(chi - cos phi)
(Section 3.3).

Static modes (Section 3.3, equation modal0):
    Ghat0_m = Q_{|m|-1/2}(chi) / (2 pi sqrt(rt r))
with Q by the three-term recurrence leg_recur started from
Q_{-1/2} = mu K(mu), Q_{1/2} = chi mu K(mu) - sqrt(2(chi+1)) E(mu),
mu = sqrt(2/(chi+1)) (K, E of modulus mu), and Q' by dleg_recur.
Static derivative modes (Section 3.3, the display after I1):
    dr Ghat0_m = Q'_{m-1/2} dr chi / (2 pi sqrt(rt r)) - Ghat0_m / (2 r),
    dz Ghat0_m = Q'_{m-1/2} dz chi / (2 pi sqrt(rt r)),
    dr chi = (r^2 - rt^2 - c^2)/(2 rt r^2),  dz chi = -c/(r rt).
k != 0 (Section 3.3, equations conv and I1, and the closing paragraph): the
derivative kernel dG/drho / rho = e^{ik rho}(ik rho - 1)/(4 pi rho^3) is split
as F * (static kernel) + i Hs with F = cos k rho + k rho sin k rho and
Hs = (k rho cos k rho - sin k rho)/(4 pi rho^3), both smooth in phi; the F part
is the convolution (1/2pi) sum_n Fhat_n X0hat_{m-n} with the static modes and
the Hs part is sampled on an equispaced grid and transformed by FFT.

Readings: Q by forward recurrence only where it is stable
(m_max acosh(chi) <= 1), otherwise Miller's backward recurrence normalised by
Q_{-1/2}; modes of the theta-dependent normal N(s, theta) are obtained by the
mode shifts m -/+ 1 of dz Ghat with weights (p' -/+ i q')/2; L_j includes the
cos N term (symmetric Nyquist, +-N halved).
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi
TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------------------
# Complete elliptic integrals by the arithmetic-geometric mean
# (Abramowitz & Stegun 17.6.3-17.6.4), modulus convention.
# ---------------------------------------------------------------------------

def ellipke(kmod, kprime):
    """K(k), E(k) for modulus k, given k and k' = sqrt(1-k^2) separately."""
    a = np.ones_like(kmod)
    b = np.array(kprime, dtype=np.float64, copy=True)
    c = np.array(kmod, dtype=np.float64, copy=True)
    s = 0.5 * c * c          # 2^{n-1} c_n^2 at n = 0
    p2 = 0.5
    for _ in range(60):
        an = 0.5 * (a + b)
        bn = np.sqrt(a * b)
        cn = c * c / (4.0 * an)       # c_n = c_{n-1}^2 / (4 a_n), free of cancellation
        a, b, c = an, bn, cn
        p2 *= 2.0
        s = s + p2 * cn * cn
        if np.all(np.abs(cn) <= 1e-17 * np.abs(a)):
            break
    K = math.pi / (2.0 * a)
    E = K * (1.0 - s)
    return K, E


def toroidal_q(chi, chim1, mmax):
    """Q[n] = Q_{n-1/2}(chi), n = 0..mmax+1, and Qp[n] = dQ_{n-1/2}/dchi, n=0..mmax.

    chi, chim1 = chi - 1 (passed separately so that chi near 1 keeps its
    digits).  Arrays of shape (P,) -> (P, mmax+2), (P, mmax+1).
    """
    chi = np.asarray(chi, dtype=np.float64)
    chim1 = np.asarray(chim1, dtype=np.float64)
    P = chi.shape[0]
    mu = np.sqrt(2.0 / (chi + 1.0))
    muprime = np.sqrt(chim1 / (chi + 1.0))
    K, E = ellipke(mu, muprime)
    q0 = mu * K
    q1 = chi * mu * K - np.sqrt(2.0 * (chi + 1.0)) * E
    nq = mmax + 2
    Q = np.zeros((P, nq))
    acosh = np.log(chi + np.sqrt(chim1 * (chi + 1.0)))
    fwd = acosh * nq <= 1.0
    # forward recurrence (stable for small m acosh chi)
    if np.any(fwd):
        idx = np.nonzero(fwd)[0]
        c = chi[idx]
        Q[idx, 0] = q0[idx]
        Q[idx, 1] = q1[idx]
        for n in range(1, nq - 1):
            Q[idx, n + 1] = (4.0 * n * c * Q[idx, n] - (2.0 * n - 1.0) * Q[idx, n - 1]) / (2.0 * n + 1.0)
    # Miller backward recurrence, normalised by Q_{-1/2}
    if np.any(~fwd):
        idx = np.nonzero(~fwd)[0]
        c = chi[idx]
        start = (nq + np.ceil(40.0 / acosh[idx]) + 10).astype(np.int64)
        nstart = int(start.max())
        hi = np.zeros(idx.shape[0])   # Q[n+1]
        lo = np.zeros(idx.shape[0])   # Q[n]
        vals = np.zeros((idx.shape[0], nq))
        for n in range(nstart, 0, -1):
            # at the start index, seed (Q[n+1], Q[n]) = (0, tiny)
            seed = start == n
            lo = np.where(seed, 1e-200, lo)
            hi = np.where(seed, 0.0, hi)
            if n < nq:
                vals[:, n] = lo
            # Q[n-1] = (4 n chi Q[n] - (2n+1) Q[n+1]) / (2n-1)
            new = (4.0 * n * c * lo - (2.0 * n + 1.0) * hi) / (2.0 * n - 1.0)
            hi, lo = lo, new
            big = np.abs(lo) > 1e200
            if np.any(big):
                sc = np.where(big, 1e-200, 1.0)
                hi = hi * sc
                lo = lo * sc
                vals = vals * sc[:, None]
        vals[:, 0] = lo
        Q[idx] = vals * (q0[idx] / lo)[:, None]
    # derivative: Q'_{n-1/2} = (2n-1)/(2(chi^2-1)) (chi Q_{n-1/2} - Q_{n-3/2}),
    # with Q_{-3/2} = Q_{1/2}
    chi2m1 = chim1 * (chi + 1.0)
    Qm1 = np.concatenate([Q[:, 1:2], Q[:, :-2]], axis=1)  # Q[n-1], n=0..mmax
    n = np.arange(mmax + 1, dtype=np.float64)
    Qp = (2.0 * n - 1.0)[None, :] / (2.0 * chi2m1[:, None]) * (chi[:, None] * Q[:, :mmax + 1] - Qm1)
    return Q, Qp


def local_frame(x, sgeo):
    """Local quantities for targets x (P,3) and source slices sgeo (dict of
    arrays r, dr, z, dz, p, dp, q, dq), from absolute coordinates.
    Returns a dict with rt, alpha, c = z_t - z, chim1 = chi - 1 and
    rmrt = r - rt (Section 3.2, equation rho2)."""
    a = x[:, 0] - sgeo["p"]
    b = x[:, 1] - sgeo["q"]
    c = x[:, 2] - sgeo["z"]
    rt = np.hypot(a, b)
    alpha = np.arctan2(b, a)
    r = sgeo["r"]
    rmrt = r - rt
    chim1 = (rmrt ** 2 + c * c) / (2.0 * r * rt)
    return dict(sgeo, rt=rt, alpha=alpha, c=c, chim1=chim1, rmrt=rmrt)


def local_frame_rel(shape, a_, c_, kappa, t, th_t, dl):
    """Same quantities for the target at parameters (t, th_t) and the source
    slice s = t + dl, using cancellation-free differences of the curve so that
    chi - 1 keeps full relative accuracy as dl -> 0."""
    from .geometry import curve, curve_differences
    r_t = curve(shape, a_, c_, kappa, t)[0]
    r, dr, z, dz, p, dp, q, dq = curve(shape, a_, c_, kappa, t + dl)
    d_r, d_z, d_p, d_q = curve_differences(shape, a_, c_, kappa, t, dl)
    ct, st = np.cos(th_t), np.sin(th_t)
    a = r_t * ct + d_p
    b = r_t * st + d_q
    rt = np.hypot(a, b)
    alpha = np.arctan2(b, a)
    drt = (2.0 * r_t * (ct * d_p + st * d_q) + d_p * d_p + d_q * d_q) / (rt + r_t)
    rmrt = d_r - drt
    c = d_z
    chim1 = (rmrt ** 2 + c * c) / (2.0 * r * rt)
    return dict(r=r, dr=dr, z=z, dz=dz, p=p, dp=dp, q=q, dq=dq,
                rt=rt, alpha=alpha, c=c, chim1=chim1, rmrt=rmrt)


def static_modes(r, rt, c, chi, chim1, mmax, rmrt=None):
    """phi-frame static modes n = 0..mmax of G, dr G, dz G (Section 3.3)."""
    Q, Qp = toroidal_q(chi, chim1, mmax)
    pref = 1.0 / (TWO_PI * np.sqrt(rt * r))
    G0 = pref[:, None] * Q[:, :mmax + 1]
    if rmrt is None:
        rmrt = r - rt
    drchi = (rmrt * (r + rt) - c * c) / (2.0 * rt * r * r)
    dzchi = -c / (r * rt)
    A0 = (pref * drchi)[:, None] * Qp - G0 / (2.0 * r)[:, None]
    B0 = (pref * dzchi)[:, None] * Qp
    return G0, A0, B0


def _rho_grid(r, rt, chim1, L):
    phi = TWO_PI * np.arange(L) / L
    s2 = np.sin(0.5 * phi) ** 2
    rho2 = 2.0 * r[:, None] * rt[:, None] * (chim1[:, None] + 2.0 * s2[None, :])
    return phi, np.sqrt(rho2)


def smooth_factor_h(k, rho):
    """Hs = (k rho cos k rho - sin k rho)/(4 pi rho^3), with its Taylor series
    (sum_{j>=1} (-1)^j 2j/(2j+1)! x^{2j+1}, x = k rho) for small k rho."""
    x = k * rho
    out = np.empty_like(rho)
    small = x < 0.5
    xs = x[small]
    ser = np.zeros_like(xs)
    term_pow = np.ones_like(xs)
    fact = 1.0
    for j in range(1, 14):
        fact = math.factorial(2 * j + 1)
        ser += ((-1) ** j) * (2.0 * j) / fact * term_pow
        term_pow = term_pow * xs * xs
    out[small] = k ** 3 / FOUR_PI * ser
    xl = x[~small]
    rl = rho[~small]
    out[~small] = (xl * np.cos(xl) - np.sin(xl)) / (FOUR_PI * rl ** 3)
    return out


def derivative_modes(k, r, rt, c, chi, chim1, nmax, L=256, nf_max=None, rmrt=None):
    """phi-frame modes n = 0..nmax of A = dr G and B = dz G for wavenumber k
    (Section 3.3): static recurrence modes, convolved with the FFT of
    F = cos k rho + k rho sin k rho, plus i times the FFT of the smooth Hs parts.
    Returns A, B of shape (P, nmax+1), complex.
    """
    P = r.shape[0]
    if k == 0.0:
        _, A0, B0 = static_modes(r, rt, c, chi, chim1, nmax, rmrt)
        return A0.astype(np.complex128), B0.astype(np.complex128)
    phi, rho = _rho_grid(r, rt, chim1, L)
    kr = k * rho
    F = np.cos(kr) + kr * np.sin(kr)
    Fh = (TWO_PI / L) * np.fft.fft(F, axis=1).real       # Fhat_n, n=0..L-1 (even)
    mag = np.abs(Fh[:, : L // 2])
    # truncation: the first index from which three consecutive |Fhat_n| lie
    # below 1e-16 max |Fhat| (Fhat decays faster than geometrically)
    low = mag < 1e-16 * mag.max(axis=1, keepdims=True)
    run = low[:, :-2] & low[:, 1:-1] & low[:, 2:]
    first = np.where(run.any(axis=1), np.argmax(run, axis=1), L // 2)
    nf = int(first.max())
    if nf_max is not None:
        nf = min(nf, nf_max)
    if nf >= L // 2 - 2:
        raise ValueError("FFT length too short for the oscillatory factor")
    _, A0, B0 = static_modes(r, rt, c, chi, chim1, nmax + nf, rmrt)
    Hs = smooth_factor_h(k, rho)
    Hr = Hs * (r[:, None] - rt[:, None] * np.cos(phi)[None, :])
    Hrh = (TWO_PI / L) * np.fft.fft(Hr, axis=1).real
    Hh = (TWO_PI / L) * np.fft.fft(Hs, axis=1).real
    A = np.zeros((P, nmax + 1), dtype=np.complex128)
    B = np.zeros((P, nmax + 1), dtype=np.complex128)
    for m in range(nmax + 1):
        accA = np.zeros(P)
        accB = np.zeros(P)
        for n in range(-nf, nf + 1):
            fn = Fh[:, abs(n)]
            idx = abs(m - n)
            accA += fn * A0[:, idx]
            accB += fn * B0[:, idx]
        A[:, m] = accA / TWO_PI + 1j * Hrh[:, m]
        B[:, m] = accB / TWO_PI + 1j * (-c) * Hh[:, m]
    return A, B


def helmholtz_modes_direct(k, r, rt, c, chim1, nmax, L=1024):
    """phi-frame modes of G, dr G, dz G by the trapezoidal rule on L points
    (definition of the modal Green's function, Section 3.1 equation
    modalgreen, and its derivatives, Section 3.2).  Only accurate when the
    kernel is smooth on the grid (chi not close to 1)."""
    phi, rho = _rho_grid(r, rt, chim1, L)
    g = np.exp(1j * k * rho) / (FOUR_PI * rho)
    dgr = np.exp(1j * k * rho) * (1j * k * rho - 1.0) / (FOUR_PI * rho ** 3)
    A = dgr * (r[:, None] - rt[:, None] * np.cos(phi)[None, :])
    B = dgr * (-c)[:, None]
    f = TWO_PI / L
    return (f * np.fft.fft(g, axis=1)[:, : nmax + 1],
            f * np.fft.fft(A, axis=1)[:, : nmax + 1],
            f * np.fft.fft(B, axis=1)[:, : nmax + 1])


def helmholtz_g_modes(k, r, rt, c, chi, chim1, nmax, L=256):
    """phi-frame modes of G itself by equation conv: I1 by convolution with the
    static modes, I2 by FFT of sin(k rho)/(4 pi rho)."""
    G0, _, _ = static_modes(r, rt, c, chi, chim1, nmax + L // 2 - 2)
    if k == 0.0:
        return G0[:, : nmax + 1].astype(np.complex128)
    phi, rho = _rho_grid(r, rt, chim1, L)
    f1 = np.cos(k * rho)
    x = k * rho
    f2 = np.where(x < 1e-8, k / FOUR_PI, np.sin(x) / (FOUR_PI * np.where(rho > 0, rho, 1.0)))
    f1h = (TWO_PI / L) * np.fft.fft(f1, axis=1).real
    f2h = (TWO_PI / L) * np.fft.fft(f2, axis=1).real
    nf = L // 2 - 2 - nmax
    out = np.zeros((r.shape[0], nmax + 1), dtype=np.complex128)
    for m in range(nmax + 1):
        acc = np.zeros(r.shape[0])
        for n in range(-nf, nf + 1):
            acc += f1h[:, abs(n)] * G0[:, abs(m - n)]
        out[:, m] = acc / TWO_PI + 1j * f2h[:, m]
    return out


# ---------------------------------------------------------------------------
# Azimuthal integrals against the trigonometric Lagrange basis
# ---------------------------------------------------------------------------

def lagrange_trig(N, theta):
    """L_j(theta), j = 0..2N-1 (Section 3.1) as an array (len(theta), 2N)."""
    thj = np.arange(2 * N) * math.pi / N
    d = np.asarray(theta)[:, None] - thj[None, :]
    out = np.ones_like(d)
    for m in range(1, N):
        out += 2.0 * np.cos(m * d)
    out += np.cos(N * d)
    return out / (2.0 * N)


def gj_modal(k, N, loc, L=256):
    """G_j(x, s) = int K(x, y(s,theta)) L_j(theta) dtheta for the double-layer
    kernel K = grad_y G . N(s, theta), N = d_theta x d_s, via modes:
    theta-frame modes K_m from phi-frame A, B (shift by e^{-i m alpha}), the
    m -/+ 1 shifts for the p' cos + q' sin part of N, then the inverse DFT
    G_j = (1/2N) sum'_{|m|<=N} K_m e^{i m theta_j} (+-N halved).
    ``loc`` is the dict returned by local_frame / local_frame_rel."""
    r, rt, c, chim1 = loc["r"], loc["rt"], loc["c"], loc["chim1"]
    A, B = derivative_modes(k, r, rt, c, 1.0 + chim1, chim1, N + 1, L=L, rmrt=loc["rmrt"])
    return _gj_from_modes(N, A, B, loc["alpha"], r, loc["dr"], loc["dz"], loc["dp"], loc["dq"])


def _gj_from_modes(N, A, B, alpha, r, dr, dz, dp, dq):
    ms = np.arange(-N, N + 1)
    absm = np.abs(ms)
    ph = np.exp(-1j * ms[None, :] * alpha[:, None])            # e^{-i m alpha}
    phm1 = np.exp(-1j * (ms - 1)[None, :] * alpha[:, None])
    php1 = np.exp(-1j * (ms + 1)[None, :] * alpha[:, None])
    Km = ph * ((r * dz)[:, None] * A[:, absm] - (r * dr)[:, None] * B[:, absm])
    Km -= (0.5 * r * (dp - 1j * dq))[:, None] * phm1 * B[:, np.abs(ms - 1)]
    Km -= (0.5 * r * (dp + 1j * dq))[:, None] * php1 * B[:, np.abs(ms + 1)]
    wts = np.ones(2 * N + 1)
    wts[0] = wts[-1] = 0.5
    thj = np.arange(2 * N) * math.pi / N
    E = np.exp(1j * ms[:, None] * thj[None, :]) * wts[:, None]   # (2N+1, 2N)
    return (Km @ E) / (2.0 * N)


def gj_sl_modal(k, N, loc, L=256):
    """G^S_j(x, s) = int G^k(x, y(s, theta)) L_j(theta) dtheta for the
    single-layer kernel G^k = e^{ik rho}/(4 pi rho) (Section 3.3, equations
    modalgreen, conv, I1): phi-frame modes of G (helmholtz_g_modes), the shift
    to the theta frame by e^{-i m alpha}, the inverse DFT as for the double
    layer (the density times |J| is what the basis interpolates)."""
    r, rt, c, chim1 = loc["r"], loc["rt"], loc["c"], loc["chim1"]
    G = helmholtz_g_modes(k, r, rt, c, 1.0 + chim1, chim1, N, L=L)
    ms = np.arange(-N, N + 1)
    Km = np.exp(-1j * ms[None, :] * loc["alpha"][:, None]) * G[:, np.abs(ms)]
    wts = np.ones(2 * N + 1)
    wts[0] = wts[-1] = 0.5
    thj = np.arange(2 * N) * math.pi / N
    E = np.exp(1j * ms[:, None] * thj[None, :]) * wts[:, None]
    return (Km @ E) / (2.0 * N)


def sl_kernel(k, x, y):
    """G^k(x, y) = e^{ik rho}/(4 pi rho) (Section 2, the Green's function)."""
    d = y - x
    rho = np.sqrt(np.sum(d * d, axis=-1))
    return np.exp(1j * k * rho) / (FOUR_PI * rho)


def gj_sl_direct(k, N, x, sgeo, L=512):
    """G^S_j by the trapezoidal rule on L azimuthal points (target away from
    the source ring)."""
    th = TWO_PI * np.arange(L) / L
    ct, st = np.cos(th)[None, :], np.sin(th)[None, :]
    g = {kk: v[:, None] for kk, v in sgeo.items()}
    y = np.stack(np.broadcast_arrays(g["r"] * ct + g["p"], g["r"] * st + g["q"], g["z"] + 0 * ct), axis=-1)
    K = sl_kernel(k, x[:, None, :], y)
    return (TWO_PI / L) * (K @ lagrange_trig(N, th))


def dl_kernel_area(k, x, y, n_area):
    """K(x, y) = grad_y G^k(x, y) . N = e^{ik rho}(ik rho - 1)/(4 pi rho^3) (y - x).N
    (Section 3.2, equations normal-derivative and dgdrho)."""
    d = y - x
    rho = np.sqrt(np.sum(d * d, axis=-1))
    return np.exp(1j * k * rho) * (1j * k * rho - 1.0) / (FOUR_PI * rho ** 3) * np.sum(d * n_area, axis=-1)


def gj_direct(k, N, x, sgeo, L=512):
    """Same G_j by the trapezoidal rule on L azimuthal points applied to the
    kernel itself (valid when the target is well away from the source ring)."""
    th = TWO_PI * np.arange(L) / L
    ct, st = np.cos(th)[None, :], np.sin(th)[None, :]
    g = {kk: v[:, None] for kk, v in sgeo.items()}
    y = np.stack(np.broadcast_arrays(g["r"] * ct + g["p"], g["r"] * st + g["q"], g["z"] + 0 * ct), axis=-1)
    ds = np.stack(np.broadcast_arrays(g["dr"] * ct + g["dp"], g["dr"] * st + g["dq"], g["dz"] + 0 * ct), axis=-1)
    dth = np.stack(np.broadcast_arrays(-g["r"] * st, g["r"] * ct, 0 * ct + 0 * g["r"]), axis=-1)
    nA = np.cross(dth, ds)
    K = dl_kernel_area(k, x[:, None, :], y, nA)   # (P, L)
    Lj = lagrange_trig(N, th)                      # (L, 2N)
    return (TWO_PI / L) * (K @ Lj)
