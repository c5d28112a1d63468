"""Pins of the oracle's naive contraction and gradient.

Oracle functions pinned: phi_naive, abar_naive, grad_naive, eval_naive.
"""

import itertools
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, lpmv

from oracle import contraction as oc
from oracle import onebody as ob
from oracle.indexsets import all_invariant_tuples, group_o3
from workloads import positions

RCUT = 5.0


def small_basis(nmax=2, lmax=2, D=4, nu=3):
    g = group_o3(nmax, lmax, D)
    return g, all_invariant_tuples(g, nu, D)


def test_ace_identity_brute_force():
    # Sec. 2.1: sum_{j1..jnu} prod_t phi_{k_t}(r_{j_t}) = prod_t sum_j phi_{k_t}(r_j)
    g, K = small_basis()
    pos = positions(3, 11)
    vals = ob.onebody_values(g.labels, pos, RCUT)   # [J, P]
    rng = np.random.default_rng(0)
    c = rng.standard_normal(len(K))
    phi = oc.eval_naive(g.labels, K, c, np.array([0, 3]), pos, RCUT)[0]
    brute = 0j
    for q, k in enumerate(K):
        s = 0j
        for js in itertools.product(range(3), repeat=len(k)):
            p = 1 + 0j
            for t, j in zip(k, js):
                p *= vals[j, t]
            s += p
        brute += c[q] * s
    assert abs(phi - brute) <= 1e-13 * max(1.0, abs(brute))


def test_single_neighbour_factorised_closed_form():
    # J = 1: A_k = prod_t R_{n_t}(r) N_{l_t m_t} P_{l_t}^{m_t}(cos th) e^{i ph sum m} and
    # sum m = 0, so phi is real and does not depend on the azimuth.  Associated
    # Legendre functions from scipy.special.lpmv (Condon-Shortley phase included).
    g, K = small_basis(3, 3, 6, 3)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(len(K))
    r, th = 2.3, 1.1

    def factor(n, l, m):
        am = abs(m)
        N = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
        P = lpmv(am, l, math.cos(th))
        val = N * P
        if m < 0:
            val *= (-1) ** am
        return math.cos(n * math.pi * r / RCUT) * val

    ref = sum(c[q] * np.prod([factor(*g.labels[i]) for i in k]) for q, k in enumerate(K))
    for ph in [0.0, 0.7, -2.5]:
        p = np.array([[r * math.sin(th) * math.cos(ph), r * math.sin(th) * math.sin(ph), r * math.cos(th)]])
        phi = oc.eval_naive(g.labels, K, c, np.array([0, 1]), p, RCUT)[0]
        assert abs(phi.imag) <= 1e-14 * max(1.0, abs(ref))
        assert abs(phi.real - ref) <= 1e-13 * max(1.0, abs(ref))


def test_single_neighbour_on_z_axis():
    # on the z axis only m_t = 0 survive: phi = sum_{k: all m = 0} c_k prod R_n sqrt((2l+1)/4pi)
    g, K = small_basis(3, 3, 6, 3)
    rng = np.random.default_rng(2)
    c = rng.standard_normal(len(K))
    r = 1.7
    ref = 0.0
    for q, k in enumerate(K):
        labs = [g.labels[i] for i in k]
        if all(m == 0 for (_, _, m) in labs):
            ref += c[q] * np.prod([math.cos(n * math.pi * r / RCUT) * math.sqrt((2 * l + 1) / (4 * math.pi))
                                   for (n, l, _) in labs])
    phi = oc.eval_naive(g.labels, K, c, np.array([0, 1]), np.array([[0.0, 0.0, r]]), RCUT)[0]
    assert abs(phi - ref) <= 1e-13 * max(1.0, abs(ref))


def test_nu2_addition_theorem_pipeline():
    # c = 2 (-1)^m on pair tuples [(n,l,m),(n',l,-m)] (1 on the diagonal tuple, 0 for
    # l != l') gives phi = sum_l (2l+1)/4pi sum_{j,j'} P_l(r_j . r_j') sum_{n,n'} R_n R_n'
    # over every ordered (n, n') with n + n' + 2l <= D (addition theorem, textbook P_l).
    nmax, lmax, D = 3, 3, 7
    g = group_o3(nmax, lmax, D)
    K = [k for k in all_invariant_tuples(g, 2, D) if len(k) == 2]
    c = np.zeros(len(K))
    for q, (i, j) in enumerate(K):
        (n1, l1, m1), (n2, l2, m2) = g.labels[i], g.labels[j]
        if l1 != l2:
            continue
        c[q] = 1.0 if i == j else 2.0 * (-1) ** m1
    pos = positions(6, 12)
    phi = oc.eval_naive(g.labels, K, c, np.array([0, 6]), pos, RCUT)[0]
    r = np.linalg.norm(pos, axis=1)
    u = pos / r[:, None]
    cosg = np.clip(u @ u.T, -1, 1)
    R = np.stack([np.cos(n * np.pi * r / RCUT) for n in range(nmax + 1)], 1)
    ref = 0.0
    for l in range(lmax + 1):
        Pl = eval_legendre(l, cosg)
        for n1 in range(nmax + 1):
            for n2 in range(nmax + 1):
                if n1 + n2 + 2 * l <= D:
                    ref += (2 * l + 1) / (4 * np.pi) * np.sum(np.outer(R[:, n1], R[:, n2]) * Pl)
    assert abs(phi.imag) <= 1e-13 * abs(ref)
    assert abs(phi.real - ref) <= 1e-12 * abs(ref)


def rot_z(a):
    return np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])


def test_invariances():
    g, K = small_basis(3, 3, 6, 3)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(len(K))
    pos = positions(9, 13)
    off = np.array([0, 9])
    phi0 = oc.eval_naive(g.labels, K, c, off, pos, RCUT)[0]
    tol = 1e-12 * max(1.0, abs(phi0))
    perm = rng.permutation(9)
    assert abs(oc.eval_naive(g.labels, K, c, off, pos[perm], RCUT)[0] - phi0) <= tol      # permutation
    assert abs(oc.eval_naive(g.labels, K, c, off, pos @ rot_z(0.83).T, RCUT)[0] - phi0) <= tol  # sum m = 0
    assert abs(oc.eval_naive(g.labels, K, c, off, -pos, RCUT)[0] - phi0) <= tol           # sum l even
    mir = pos * np.array([1, 1, -1])
    assert abs(oc.eval_naive(g.labels, K, c, off, mir, RCUT)[0] - phi0) <= tol            # z -> -z
    # a full rotation is *not* a symmetry for generic c (the check is not vacuous)
    Q = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    assert abs(oc.eval_naive(g.labels, K, c, off, pos @ Q.T, RCUT)[0] - phi0) > 1e-6 * abs(phi0)


def test_abar_brute_force_and_euler_identity():
    g, K = small_basis(2, 2, 4, 3)
    rng = np.random.default_rng(4)
    c = rng.standard_normal(len(K))
    A = rng.standard_normal((2, len(g))) + 1j * rng.standard_normal((2, len(g)))
    Ab = oc.abar_naive(K, c, A)
    # holomorphic derivative by complex-step-free brute force: phi is a polynomial,
    # so d phi/dA_i = (phi(A + h e_i) - phi(A - h e_i)) / 2h exactly up to O(h^2) * 3rd derivative
    h = 1e-5
    for i in range(len(g)):
        Ap, Am = A.copy(), A.copy()
        Ap[:, i] += h
        Am[:, i] -= h
        fd = (oc.phi_naive(K, c, Ap) - oc.phi_naive(K, c, Am)) / (2 * h)
        np.testing.assert_allclose(Ab[:, i], fd, rtol=1e-7, atol=1e-8)
    # Euler: each term is homogeneous of degree nu(k): sum_i A_i Abar_i = sum_k nu(k) c_k A_k
    lhs = np.sum(A * Ab, axis=1)
    rhs = oc.phi_naive(K, c * np.array([len(k) for k in K]), A)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_gradient_finite_differences_and_symmetries():
    g, K = small_basis(3, 3, 6, 3)
    rng = np.random.default_rng(5)
    c = rng.standard_normal(len(K))
    pos = positions(10, 14)
    off = np.array([0, 4, 10])
    phi, G = oc.grad_naive(g.labels, K, c, off, pos, RCUT)
    h = 1e-6
    fd = np.zeros_like(pos)
    for j in range(len(pos)):
        for d in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[j, d] += h
            p2[j, d] -= h
            e = 0 if j < 4 else 1
            fd[j, d] = (oc.eval_naive(g.labels, K, c, off, p1, RCUT)[e].real
                        - oc.eval_naive(g.labels, K, c, off, p2, RCUT)[e].real) / (2 * h)
    assert np.linalg.norm(G - fd) <= 1e-7 * np.linalg.norm(G)
    # invariance under rotation about z => zero z-torque per environment
    for a, b in [(0, 4), (4, 10)]:
        tz = np.sum(pos[a:b, 0] * G[a:b, 1] - pos[a:b, 1] * G[a:b, 0])
        assert abs(tz) <= 1e-12 * np.abs(G).sum()
    # inversion: g(-r) = -g(r)
    _, G2 = oc.grad_naive(g.labels, K, c, off, -pos, RCUT)
    np.testing.assert_allclose(G2, -G, atol=1e-12 * np.abs(G).max())
    # covariance under rotation about z: g(Q r) = Q g(r)
    Q = rot_z(-1.1)
    _, G3 = oc.grad_naive(g.labels, K, c, off, pos @ Q.T, RCUT)
    np.testing.assert_allclose(G3, G @ Q.T, atol=1e-12 * np.abs(G).max())


def test_empty_environment_and_nu1():
    g, K = small_basis(2, 2, 4, 2)
    c = np.ones(len(K))
    pos = positions(3, 15)
    phi = oc.eval_naive(g.labels, K, c, np.array([0, 0, 3]), pos, RCUT)
    assert phi[0] == 0
    # nu = 1 only: phi = sum_{i: m=0, l even} A_i
    K1 = [k for k in K if len(k) == 1]
    A = ob.pooled_A(g.labels, np.array([0, 3]), pos, RCUT)[0]
    ref = sum(A[k[0]] for k in K1)
    got = oc.eval_naive(g.labels, K1, np.ones(len(K1)), np.array([0, 3]), pos, RCUT)[0]
    assert abs(got - ref) <= 1e-14 * abs(ref)


def test_stored_oracle_samples_reproduce():
    """The stored oracle values of the 32768-environment workload (written by
    tests/golden/make_oracle_samples.py) match their inputs' fingerprint and a
    live oracle run on two of their environments (the smallest and the largest
    neighbour count)."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    from make_oracle_samples import fingerprint, path_for
    import workloads as wl
    from oracle.contraction import grad_naive
    from oracle.indexsets import all_invariant_tuples, group_o3
    w = wl.WORKLOADS[4]
    g = group_o3(w.n_max, w.l_max, w.degree_max)
    K = all_invariant_tuples(g, w.nu_max, w.degree_max)
    c = wl.coefficients(w, np.array([g.degree(k) for k in K]))
    off, pos = wl.batch(w)
    d = np.load(path_for(4))
    envs = d["envs"]
    so, sp_ = wl.gather(off, pos, envs)
    assert np.array_equal(so, d["offsets"]) and str(d["fingerprint"]) == fingerprint(sp_, c)
    J = np.diff(off)
    for e in (int(envs[np.argmin(J[envs])]), int(envs[np.argmax(J[envs])])):
        i = int(np.nonzero(envs == e)[0][0])
        o1, p1 = wl.gather(off, pos, [e])
        phi, grad = grad_naive(g.labels, K, c, o1, p1, w.r_cut)
        assert abs(phi[0] - d["phi"][i]) <= 1e-13 * abs(phi[0])
        rows = slice(int(so[i]), int(so[i + 1]))
        assert np.allclose(grad, d["grad"][rows], rtol=1e-12, atol=1e-14 * np.abs(grad).max())
