"""Pins of the oracle's one-particle basis: closed forms, textbook identities,
an arbitrary-precision library, and finite differences.

Oracle functions pinned: chebyshev_T, chebyshev_U, radial, radial_deriv,
ylm, onebody_values, onebody_gradients, pooled_A.
"""

import math

import mpmath
import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle import onebody as ob
from workloads import positions

RCUT = 5.0


def test_radial_closed_form():
    # T_n(cos t) = cos(n t) with t = pi r / r_cut in (0.1 pi, pi) on the shell
    r = np.linspace(0.5, 4.999, 101)
    R = ob.radial(10, r, RCUT)
    for n in range(11):
        np.testing.assert_allclose(R[:, n], np.cos(n * np.pi * r / RCUT), rtol=0, atol=2e-14)


def test_radial_derivative_closed_form():
    r = np.linspace(0.5, 4.999, 101)
    dR = ob.radial_deriv(10, r, RCUT)
    for n in range(11):
        ref = -(n * np.pi / RCUT) * np.sin(n * np.pi * r / RCUT)
        np.testing.assert_allclose(dR[:, n], ref, rtol=0, atol=1e-12)


def test_chebyshev_U_closed_form():
    t = np.linspace(0.1, 3.0, 37)
    U = ob.chebyshev_U(8, np.cos(t))
    for n in range(9):
        np.testing.assert_allclose(U[:, n], np.sin((n + 1) * t) / np.sin(t), atol=1e-12)


def test_ylm_explicit_low_orders():
    rng = np.random.default_rng(3)
    th = rng.uniform(0.05, np.pi - 0.05, 20)
    ph = rng.uniform(-np.pi, np.pi, 20)
    s, c = np.sin(th), np.cos(th)
    pi = np.pi
    np.testing.assert_allclose(ob.ylm(0, 0, th, ph), np.full(20, 1 / math.sqrt(4 * pi)), atol=1e-15)
    np.testing.assert_allclose(ob.ylm(1, 0, th, ph), math.sqrt(3 / (4 * pi)) * c, atol=1e-15)
    np.testing.assert_allclose(ob.ylm(1, 1, th, ph), -math.sqrt(3 / (8 * pi)) * s * np.exp(1j * ph), atol=1e-15)
    np.testing.assert_allclose(ob.ylm(1, -1, th, ph), math.sqrt(3 / (8 * pi)) * s * np.exp(-1j * ph), atol=1e-15)
    np.testing.assert_allclose(ob.ylm(2, 0, th, ph), math.sqrt(5 / (16 * pi)) * (3 * c * c - 1), atol=1e-15)
    np.testing.assert_allclose(ob.ylm(2, 1, th, ph), -math.sqrt(15 / (8 * pi)) * s * c * np.exp(1j * ph), atol=1e-15)
    np.testing.assert_allclose(ob.ylm(2, 2, th, ph), 0.25 * math.sqrt(15 / (2 * pi)) * s * s * np.exp(2j * ph),
                               atol=1e-15)


def test_ylm_addition_theorem_and_conjugation():
    rng = np.random.default_rng(4)
    u = rng.standard_normal((30, 3))
    v = rng.standard_normal((30, 3))
    _, tu, pu = ob.spherical_coords(u)
    _, tv, pv = ob.spherical_coords(v)
    cosg = np.sum(u * v, 1) / np.linalg.norm(u, axis=1) / np.linalg.norm(v, axis=1)
    for l in range(11):
        s_norm = sum(np.abs(ob.ylm(l, m, tu, pu)) ** 2 for m in range(-l, l + 1))
        np.testing.assert_allclose(s_norm, (2 * l + 1) / (4 * np.pi), rtol=1e-13)
        s_add = sum(ob.ylm(l, m, tu, pu) * np.conj(ob.ylm(l, m, tv, pv)) for m in range(-l, l + 1))
        np.testing.assert_allclose(s_add, (2 * l + 1) / (4 * np.pi) * eval_legendre(l, cosg), atol=1e-13)
        for m in range(0, l + 1):
            np.testing.assert_allclose(ob.ylm(l, -m, tu, pu), (-1) ** m * np.conj(ob.ylm(l, m, tu, pu)), atol=1e-14)


def test_ylm_orthonormal_by_quadrature():
    x, w = np.polynomial.legendre.leggauss(24)
    th = np.arccos(x)
    nph = 32
    ph = 2 * np.pi * np.arange(nph) / nph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(w, np.full(nph, 2 * np.pi / nph))
    idx = [(l, m) for l in range(7) for m in range(-l, l + 1)]
    Y = np.stack([ob.ylm(l, m, TH, PH) for (l, m) in idx])
    G = np.einsum("aij,bij,ij->ab", Y, np.conj(Y), W)
    np.testing.assert_allclose(G, np.eye(len(idx)), atol=1e-13)


def test_ylm_against_mpmath():
    rng = np.random.default_rng(5)
    mpmath.mp.dps = 30
    for _ in range(12):
        l = int(rng.integers(0, 11))
        m = int(rng.integers(-l, l + 1))
        th = float(rng.uniform(0.1, 3.0))
        ph = float(rng.uniform(-3.0, 3.0))
        ref = complex(mpmath.spherharm(l, m, th, ph))
        got = complex(ob.ylm(l, m, np.array([th]), np.array([ph]))[0])
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))


LABELS = [(n, l, m) for n in range(4) for l in range(5) for m in range(-l, l + 1) if n + l <= 7]


def test_onebody_gradient_central_differences():
    pos = positions(8, 91)
    g = ob.onebody_gradients(LABELS, pos, RCUT)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (ob.onebody_values(LABELS, pos + e, RCUT) - ob.onebody_values(LABELS, pos - e, RCUT)) / (2 * h)
        np.testing.assert_allclose(g[:, :, d], fd, atol=2e-8)


def test_onebody_gradient_high_precision_fd():
    # mpmath finite differences of R_n Y_l^m at 40 digits for a few functions
    mpmath.mp.dps = 40
    r0 = np.array([[1.3, -0.7, 2.1]])
    lab = [(2, 3, -2), (0, 4, 3), (3, 1, 0)]
    g = ob.onebody_gradients(lab, r0, RCUT)[0]

    def f(i, x, y, z):
        n, l, m = lab[i]
        r = mpmath.sqrt(x * x + y * y + z * z)
        th = mpmath.acos(z / r)
        ph = mpmath.atan2(y, x)
        return mpmath.cos(n * mpmath.pi * r / RCUT) * mpmath.spherharm(l, m, th, ph)

    for i in range(len(lab)):
        for d in range(3):
            def fd(t, i=i, d=d):
                p = [mpmath.mpf(v) for v in r0[0]]
                p[d] += t
                return f(i, *p)
            ref = complex(mpmath.diff(fd, 0))
            assert abs(g[i, d] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_ylm_gradient_is_tangential():
    pos = positions(16, 92)
    g = ob.onebody_gradients([(0, l, m) for l in range(6) for m in range(-l, l + 1)], pos, RCUT)
    radial_part = np.einsum("jid,jd->ji", g, pos)
    np.testing.assert_allclose(radial_part, 0, atol=1e-13)


def test_pooled_A_is_sum_over_neighbours():
    pos = positions(7, 93)
    off = np.array([0, 3, 3, 7])
    A = ob.pooled_A(LABELS, off, pos, RCUT)
    vals = ob.onebody_values(LABELS, pos, RCUT)
    np.testing.assert_allclose(A[0], vals[0] + vals[1] + vals[2], atol=1e-15)
    assert np.all(A[1] == 0)
    np.testing.assert_allclose(A[2], vals[3:7].sum(0), atol=1e-15)


def test_onebody_values_near_the_poles_against_mpmath():
    """Positions on and within 1e-12..1e-4 of the z-axis: the one-particle values
    against mpmath (40 digits) from the exact spherical angles of the same
    binary64 coordinates.  Computing the polar angle as arccos(z / r) would
    lose about 1e-16 / theta^2 relative accuracy here."""
    mpmath.mp.dps = 40
    labels = [(n, l, m) for n in range(3) for l in range(5) for m in range(-l, l + 1)]
    rng = np.random.default_rng(5)
    pts = []
    for sign in (1.0, -1.0):
        for delta in (0.0, 1e-12, 1e-8, 1e-6, 1e-4):
            r, beta = rng.uniform(1.0, 4.5), rng.uniform(-np.pi, np.pi)
            pts.append(r * np.array([math.sin(delta) * math.cos(beta), math.sin(delta) * math.sin(beta),
                                     sign * math.cos(delta)]))
    pos = np.array(pts)
    vals = ob.onebody_values(labels, pos, 5.0)
    for j, p in enumerate(pos):
        x, y, z = (mpmath.mpf(float(v)) for v in p)
        rr = mpmath.sqrt(x * x + y * y + z * z)
        th = mpmath.atan2(mpmath.sqrt(x * x + y * y), z)
        ph = mpmath.atan2(y, x)
        for i, (n, l, m) in enumerate(labels):
            ref = complex(mpmath.cos(n * mpmath.pi * rr / 5) * mpmath.spherharm(l, m, th, ph))
            scale = math.sqrt((2 * l + 1) / (4 * math.pi))
            assert abs(vals[j, i] - ref) <= 1e-14 * scale, (j, n, l, m)
