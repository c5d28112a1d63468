"""One-particle bases, pooled A, gradients: O(3) phi_nlm(r) = R_n(|r|) Y_l^m(r/|r|);
the planar groups of Sec. 2.2 and 2.3 (torus e^{i m theta}, SO(2) R_n(r) e^{-i m theta}).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed:
  * phi_nlm(r) = R_n(r) Y_l^m(r_hat), standard complex spherical harmonics
    (Sec. 2.4);  A_k = sum_j phi_k(r_j)  (Sec. 2.1, Eq. (2.1)).
  * The radial basis is "not essential" (Sec. 2.6); the workloads use
    R_n(r) = T_n(cos(pi r / r_cut)), Chebyshev polynomials of the first kind,
    n = 0..n_max.
Convention for Y (the paper says only "standard complex"): orthonormal on
the sphere, Condon-Shortley phase, azimuthal factor e^{+i m phi}, which is
what scipy.special.sph_harm_y returns.

Route of the derivatives (independent of any Cartesian recurrence):
  dR_n/dr = T_n'(x) dx/dr,  T_n' = n U_{n-1}  (Chebyshev U by recurrence)
  dY/dphi = i m Y
  dY/dtheta = m cot(theta) Y_l^m + sqrt((l-m)(l+m+1)) e^{-i phi} Y_l^{m+1}
  grad Y(r) = (theta_hat dY/dtheta + phi_hat dY/dphi / sin(theta)) / |r|
The formulas divide by sin(theta); the oracle is only used on random
directions, where theta is bounded away from 0 and pi.
"""

from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y


def chebyshev_T(nmax: int, x: np.ndarray) -> np.ndarray:
    """T_0..T_nmax at x by T_{n+1} = 2 x T_n - T_{n-1}; shape x.shape + (nmax+1,)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape + (nmax + 1,))
    out[..., 0] = 1.0
    if nmax >= 1:
        out[..., 1] = x
    for n in range(1, nmax):
        out[..., n + 1] = 2.0 * x * out[..., n] - out[..., n - 1]
    return out


def chebyshev_U(nmax: int, x: np.ndarray) -> np.ndarray:
    """U_0..U_nmax at x by U_{n+1} = 2 x U_n - U_{n-1}, U_0 = 1, U_1 = 2x."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape + (nmax + 1,))
    out[..., 0] = 1.0
    if nmax >= 1:
        out[..., 1] = 2.0 * x
    for n in range(1, nmax):
        out[..., n + 1] = 2.0 * x * out[..., n] - out[..., n - 1]
    return out


def radial(nmax: int, r: np.ndarray, r_cut: float) -> np.ndarray:
    """R_n(r) = T_n(cos(pi r / r_cut)), n = 0..nmax."""
    return chebyshev_T(nmax, np.cos(np.pi * np.asarray(r) / r_cut))


def radial_deriv(nmax: int, r: np.ndarray, r_cut: float) -> np.ndarray:
    """dR_n/dr = n U_{n-1}(x) * dx/dr with x = cos(pi r / r_cut)."""
    r = np.asarray(r, dtype=np.float64)
    x = np.cos(np.pi * r / r_cut)
    dxdr = -(np.pi / r_cut) * np.sin(np.pi * r / r_cut)
    U = chebyshev_U(max(nmax - 1, 0), x)
    out = np.zeros(r.shape + (nmax + 1,))
    for n in range(1, nmax + 1):
        out[..., n] = n * U[..., n - 1] * dxdr
    return out


def spherical_coords(pos: np.ndarray):
    """|r|, polar angle theta in [0, pi], azimuth phi in (-pi, pi].

    theta = atan2(sqrt(x^2 + y^2), z): the same angle as arccos(z / r), which
    loses accuracy within a few degrees of the z-axis (its error grows like
    eps / theta^2), whereas this form keeps full relative accuracy there."""
    pos = np.asarray(pos, dtype=np.float64)
    r = np.sqrt(np.sum(pos * pos, axis=-1))
    theta = np.arctan2(np.hypot(pos[..., 0], pos[..., 1]), pos[..., 2])
    phi = np.arctan2(pos[..., 1], pos[..., 0])
    return r, theta, phi


def ylm(l: int, m: int, theta, phi):
    """Complex orthonormal Y_l^m (Condon-Shortley, e^{+i m phi}); 0 if |m| > l."""
    if abs(m) > l:
        return np.zeros(np.broadcast(theta, phi).shape, dtype=np.complex128)
    return sph_harm_y(l, m, theta, phi)


def _planar(labels) -> bool:
    """Torus labels are integers m, SO(2) labels pairs (n, m), O(3) labels triples
    (quadruples with a feature)."""
    return len(labels) > 0 and (not isinstance(labels[0], tuple) or len(labels[0]) == 2)


def planar_values(labels, pos: np.ndarray, r_cut: float) -> np.ndarray:
    """Planar one-particle functions at r_j = (x_j, y_j) (z ignored), with
    theta = atan2(y, x) and r = |(x, y)|; [J, P1]:
      torus (Sec. 2.3): phi_m = e^{+i m theta};
      SO(2) (Sec. 2.2): phi_nm = R_n(r) e^{-i m theta}."""
    pos = np.asarray(pos, dtype=np.float64)
    th = np.arctan2(pos[:, 1], pos[:, 0])
    out = np.empty((pos.shape[0], len(labels)), dtype=np.complex128)
    if not isinstance(labels[0], tuple):
        for i, m in enumerate(labels):
            out[:, i] = np.exp(1j * m * th)
        return out
    r = np.hypot(pos[:, 0], pos[:, 1])
    R = radial(max(n for (n, _) in labels), r, r_cut)
    for i, (n, m) in enumerate(labels):
        out[:, i] = R[:, n] * np.exp(-1j * m * th)
    return out


def planar_gradients(labels, pos: np.ndarray, r_cut: float) -> np.ndarray:
    """grad phi_i(r_j) of the planar functions; complex [J, P1, 3], z part 0.
    grad theta = (-y, x) / r^2, grad r = (x, y) / r."""
    pos = np.asarray(pos, dtype=np.float64)
    x, y = pos[:, 0], pos[:, 1]
    r2 = x * x + y * y
    r = np.sqrt(r2)
    th = np.arctan2(y, x)
    gth = np.stack([-y / r2, x / r2, np.zeros_like(x)], axis=-1)
    grr = np.stack([x / r, y / r, np.zeros_like(x)], axis=-1)
    out = np.empty((pos.shape[0], len(labels), 3), dtype=np.complex128)
    if not isinstance(labels[0], tuple):
        for i, m in enumerate(labels):
            out[:, i, :] = (1j * m * np.exp(1j * m * th))[:, None] * gth
        return out
    nmax = max(n for (n, _) in labels)
    R = radial(nmax, r, r_cut)
    dR = radial_deriv(nmax, r, r_cut)
    for i, (n, m) in enumerate(labels):
        e = np.exp(-1j * m * th)
        out[:, i, :] = (dR[:, n] * e)[:, None] * grr + (R[:, n] * (-1j * m) * e)[:, None] * gth
    return out


def _features(labels) -> bool:
    return len(labels) > 0 and isinstance(labels[0], tuple) and len(labels[0]) == 4


def feature_values(labels, pos: np.ndarray, r_cut: float) -> np.ndarray:
    """Sec. 5.4: phi_nlmk(r, mu) = R_n(r) Y_l^m(r_hat) T_k(mu); positions carry
    the feature as a fourth column, pos [J, 4] = (x, y, z, mu); [J, P1]."""
    pos = np.asarray(pos, dtype=np.float64)
    base_lab = sorted({(n, l, m) for (n, l, m, _) in labels})
    base = onebody_values(base_lab, pos[:, :3], r_cut)
    col = {t: i for i, t in enumerate(base_lab)}
    Tk = chebyshev_T(max(k for (*_, k) in labels), pos[:, 3])
    out = np.empty((pos.shape[0], len(labels)), dtype=np.complex128)
    for i, (n, l, m, k) in enumerate(labels):
        out[:, i] = base[:, col[(n, l, m)]] * Tk[:, k]
    return out


def feature_gradients(labels, pos: np.ndarray, r_cut: float) -> np.ndarray:
    """grad over the position (the feature is a label): T_k(mu) grad(R_n Y_l^m);
    complex [J, P1, 3]."""
    pos = np.asarray(pos, dtype=np.float64)
    base_lab = sorted({(n, l, m) for (n, l, m, _) in labels})
    base = onebody_gradients(base_lab, pos[:, :3], r_cut)
    col = {t: i for i, t in enumerate(base_lab)}
    Tk = chebyshev_T(max(k for (*_, k) in labels), pos[:, 3])
    out = np.empty((pos.shape[0], len(labels), 3), dtype=np.complex128)
    for i, (n, l, m, k) in enumerate(labels):
        out[:, i, :] = base[:, col[(n, l, m)], :] * Tk[:, k][:, None]
    return out


def onebody_values(labels, pos: np.ndarray, r_cut: float) -> np.ndarray:
    """phi_i(r_j) for every one-particle label; [J, P1].  O(3) triples (n, l, m);
    torus and SO(2) labels go to planar_values, O(3) with a feature (n, l, m, k)
    to feature_values."""
    if _planar(labels):
        return planar_values(labels, pos, r_cut)
    if _features(labels):
        return feature_values(labels, pos, r_cut)
    r, th, ph = spherical_coords(pos)
    nmax = max(n for (n, _, _) in labels)
    R = radial(nmax, r, r_cut)
    cache = {}
    out = np.empty((len(r), len(labels)), dtype=np.complex128)
    for i, (n, l, m) in enumerate(labels):
        if (l, m) not in cache:
            cache[(l, m)] = ylm(l, m, th, ph)
        out[:, i] = R[:, n] * cache[(l, m)]
    return out


def onebody_gradients(labels, pos: np.ndarray, r_cut: float) -> np.ndarray:
    """grad_r phi_i(r_j); complex [J, P1, 3], by the spherical-coordinate route
    (torus and SO(2) labels go to planar_gradients)."""
    if _planar(labels):
        return planar_gradients(labels, pos, r_cut)
    if _features(labels):
        return feature_gradients(labels, pos, r_cut)
    pos = np.asarray(pos, dtype=np.float64)
    r, th, ph = spherical_coords(pos)
    nmax = max(n for (n, _, _) in labels)
    R = radial(nmax, r, r_cut)
    dR = radial_deriv(nmax, r, r_cut)
    st, ct = np.sin(th), np.cos(th)
    sp, cp = np.sin(ph), np.cos(ph)
    rhat = pos / r[:, None]
    that = np.stack([ct * cp, ct * sp, -st], axis=-1)
    phat = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    Ycache = {}

    def Y(l, m):
        if (l, m) not in Ycache:
            Ycache[(l, m)] = ylm(l, m, th, ph)
        return Ycache[(l, m)]

    gcache = {}

    def gradY(l, m):
        if (l, m) not in gcache:
            y = Y(l, m)
            dth = m * (ct / st) * y
            if m + 1 <= l:
                dth = dth + np.sqrt((l - m) * (l + m + 1)) * np.exp(-1j * ph) * Y(l, m + 1)
            dph = 1j * m * y
            g = (that * dth[:, None] + phat * (dph / st)[:, None]) / r[:, None]
            gcache[(l, m)] = g
        return gcache[(l, m)]

    out = np.empty((len(r), len(labels), 3), dtype=np.complex128)
    for i, (n, l, m) in enumerate(labels):
        out[:, i, :] = (dR[:, n] * Y(l, m))[:, None] * rhat + R[:, n][:, None] * gradY(l, m)
    return out


def pooled_A(labels, offsets: np.ndarray, pos: np.ndarray, r_cut: float) -> np.ndarray:
    """A[e, i] = sum_{j in env e} phi_i(r_j)  (Sec. 2.1, Eq. (2.1)); [E, P1]."""
    offsets = np.asarray(offsets)
    E = len(offsets) - 1
    vals = onebody_values(labels, pos, r_cut)
    A = np.zeros((E, len(labels)), dtype=np.complex128)
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        if b > a:
            A[e] = vals[a:b].sum(axis=0)
    return A
