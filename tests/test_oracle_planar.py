"""Pins of the oracle's planar groups (Sec. 2.2 SO(2), Sec. 2.3 torus): index
sets by brute force, one-particle values by an algebraic route, gradients by
central differences, the symmetries of Sec. 2.2, a single-neighbour closed form
and the ACE identity."""

import itertools

import numpy as np
import pytest

import workloads as wl
from oracle import contraction as oc
from oracle import onebody as ob
from oracle.indexsets import all_invariant_tuples, group_so2, group_torus, invariant_tuples


def planar_positions(n, seed, r_lo=0.5, r_hi=5.0):
    g = np.random.default_rng(seed)
    th = g.uniform(-np.pi, np.pi, n)
    r = g.uniform(r_lo, r_hi, n)
    z = g.standard_normal(n)          # ignored by the planar bases
    return np.stack([r * np.cos(th), r * np.sin(th), z], axis=-1)


def test_so2_onebody_list():
    lab = group_so2(2, 2, 3).labels
    assert lab[:4] == [(0, 0), (1, 0), (0, -1), (0, 1)]
    assert all(n + abs(m) <= 3 and n <= 2 and abs(m) <= 2 for (n, m) in lab)
    assert len(lab) == len(set(lab)) == 13


@pytest.mark.parametrize("nu", [1, 2, 3, 4])
def test_so2_K_matches_brute_force(nu):
    g = group_so2(2, 3, 5)
    brute = [t for t in itertools.combinations_with_replacement(range(len(g)), nu)
             if sum(g.m[i] for i in t) == 0 and g.degree(t) <= 5]
    assert invariant_tuples(g, nu, 5) == brute


def test_planar_values_by_complex_powers():
    # e^{-i m theta} = ((x - i y) / r)^m for m >= 0 and ((x + i y) / r)^{|m|} for m < 0
    pos = planar_positions(40, 1)
    x, y = pos[:, 0], pos[:, 1]
    r = np.hypot(x, y)
    u = (x - 1j * y) / r
    g = group_so2(3, 4, 6)
    R = np.cos(np.outer(np.pi * r / 5.0, np.arange(4)))   # T_n(cos a) = cos(n a)
    ref = np.stack([R[:, n] * (u ** m if m >= 0 else np.conj(u) ** (-m)) for (n, m) in g.labels], axis=1)
    assert np.allclose(ob.onebody_values(g.labels, pos, 5.0), ref, rtol=0, atol=1e-13)
    t = group_torus(4)
    reft = np.stack([np.conj(u) ** m if m >= 0 else u ** (-m) for m in t.labels], axis=1)
    assert np.allclose(ob.onebody_values(t.labels, pos, 5.0), reft, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind", ["so2", "torus"])
def test_planar_gradients_central_differences(kind):
    g = group_so2(3, 3, 5) if kind == "so2" else group_torus(5)
    pos = planar_positions(12, 2)
    G = ob.onebody_gradients(g.labels, pos, 5.0)
    h = 1e-6
    for d in range(3):
        pp, pm = pos.copy(), pos.copy()
        pp[:, d] += h
        pm[:, d] -= h
        fd = (ob.onebody_values(g.labels, pp, 5.0) - ob.onebody_values(g.labels, pm, 5.0)) / (2 * h)
        assert np.allclose(G[:, :, d], fd, rtol=1e-7, atol=1e-7)
    assert np.all(G[:, :, 2] == 0)


def _phi(g, K, c, off, pos):
    return oc.eval_naive(g.labels, K, c, off, pos, 5.0)


@pytest.mark.parametrize("kind", ["so2", "torus"])
def test_rotation_invariance_and_reflection_conjugates(kind):
    g = group_so2(3, 3, 6) if kind == "so2" else group_torus(6)
    K = all_invariant_tuples(g, 4, 6)
    c = np.random.default_rng(3).standard_normal(len(K))
    off = np.array([0, 4, 9, 16], np.int32)
    pos = planar_positions(16, 4)
    phi = _phi(g, K, c, off, pos)
    a = 0.83
    Q = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    assert np.allclose(_phi(g, K, c, off, pos @ Q.T), phi, rtol=1e-12, atol=1e-12)
    # Sec. 2.2: a reflection conjugates every invariant A_k, so Re phi is O(2)-invariant
    refl = pos * np.array([1.0, -1.0, 1.0])
    assert np.allclose(_phi(g, K, c, off, refl), np.conj(phi), rtol=1e-12, atol=1e-12)
    assert np.abs(phi.imag).max() > 1e-3


def test_so2_single_neighbour_closed_form():
    # one neighbour: A_k = prod_t R_{n_t}(r) e^{-i theta sum m} = prod_t R_{n_t}(r), real
    g = group_so2(4, 3, 6)
    K = all_invariant_tuples(g, 3, 6)
    c = np.random.default_rng(5).standard_normal(len(K))
    pos = planar_positions(1, 6)
    r = np.hypot(pos[0, 0], pos[0, 1])
    Rn = np.cos(np.pi * r / 5.0 * np.arange(5))
    ref = sum(ck * np.prod([Rn[g.labels[i][0]] for i in k]) for ck, k in zip(c, K))
    phi = _phi(g, K, c, np.array([0, 1]), pos)
    assert abs(phi[0] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_planar_ace_identity_brute_force():
    # A_k = sum over all neighbour tuples of prod_t phi_{k_t}(r_{j_t})  (Sec. 2.1)
    g = group_so2(2, 2, 4)
    pos = planar_positions(3, 7)
    vals = ob.onebody_values(g.labels, pos, 5.0)
    A = vals.sum(axis=0)
    for k in all_invariant_tuples(g, 3, 4)[:40]:
        brute = sum(np.prod([vals[j, i] for j, i in zip(js, k)]) for js in itertools.product(range(3), repeat=len(k)))
        assert abs(np.prod(A[list(k)]) - brute) <= 1e-12 * max(1.0, abs(brute))


def test_planar_gradient_of_phi_central_differences():
    g = group_so2(3, 3, 6)
    K = all_invariant_tuples(g, 3, 6)
    c = np.random.default_rng(8).standard_normal(len(K))
    off = np.array([0, 5], np.int32)
    pos = planar_positions(5, 9)
    _, grad = oc.grad_naive(g.labels, K, c, off, pos, 5.0)
    h = 1e-6
    fd = np.zeros_like(pos)
    for j in range(5):
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[j, d] += h
            pm[j, d] -= h
            fd[j, d] = (_phi(g, K, c, off, pp)[0].real - _phi(g, K, c, off, pm)[0].real) / (2 * h)
    assert np.allclose(grad, fd, rtol=1e-6, atol=1e-7)
