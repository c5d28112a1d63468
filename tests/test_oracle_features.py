"""Pins of the oracle's invariant-feature basis (Sec. 5.4):
phi_nlmk(r, mu) = R_n(r) Y_l^m(r_hat) T_k(mu), degree n + l + k."""

import itertools

import numpy as np
import pytest

from oracle import contraction as oc
from oracle import onebody as ob
from oracle.indexsets import (all_invariant_tuples, group_o3, group_o3_features, invariant_tuples,
                              onebody_o3_features)


def shell_positions(n, seed, mu=None):
    g = np.random.default_rng(seed)
    d = g.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = g.uniform(0.5, 5.0, n)
    m = g.uniform(-1, 1, n) if mu is None else np.full(n, mu)
    return np.concatenate([d * r[:, None], m[:, None]], axis=1)


def test_feature_list_order_and_reduction():
    lab = onebody_o3_features(2, 2, 2, 4)
    assert len(lab) == len(set(lab))
    assert all(n + l + k <= 4 and abs(m) <= l for (n, l, m, k) in lab)
    key = [(n + l + k, l, k, m) for (n, l, m, k) in lab]
    assert key == sorted(key)
    # the 2l+1 functions of one (n, l, k) are consecutive
    for (n, l, m, k) in lab:
        if m == -l:
            i = lab.index((n, l, m, k))
            assert lab[i:i + 2 * l + 1] == [(n, l, mm, k) for mm in range(-l, l + 1)]
    # k_max = 0 is the plain O(3) list
    assert [(n, l, m) for (n, l, m, _) in onebody_o3_features(3, 3, 0, 5)] == group_o3(3, 3, 5).labels


@pytest.mark.parametrize("nu", [1, 2, 3])
def test_feature_K_matches_brute_force(nu):
    g = group_o3_features(1, 2, 2, 4)
    brute = [t for t in itertools.combinations_with_replacement(range(len(g)), nu)
             if g.is_invariant(t) and g.degree(t) <= 4]
    assert invariant_tuples(g, nu, 4) == brute


def test_feature_values_reduce_to_o3_when_mu_is_one():
    # T_k(1) = 1: every k copies the plain O(3) function
    g = group_o3_features(3, 3, 2, 6)
    pos = shell_positions(30, 1, mu=1.0)
    v = ob.onebody_values(g.labels, pos, 5.0)
    base = group_o3(3, 3, 6)
    vb = ob.onebody_values(base.labels, pos[:, :3], 5.0)
    col = {t: i for i, t in enumerate(base.labels)}
    for i, (n, l, m, k) in enumerate(g.labels):
        assert np.allclose(v[:, i], vb[:, col[(n, l, m)]], rtol=0, atol=1e-14)


def test_feature_chebyshev_by_cosines():
    # T_k(cos a) = cos(k a), an independent route for the feature polynomials
    g = group_o3_features(0, 0, 5, 5)      # only l = n = 0: phi = Y_0^0 T_k(mu)
    a = np.random.default_rng(2).uniform(0, np.pi, 20)
    pos = shell_positions(20, 3)
    pos[:, 3] = np.cos(a)
    v = ob.onebody_values(g.labels, pos, 5.0)
    y00 = 1.0 / np.sqrt(4 * np.pi)
    R0 = 1.0
    for i, (n, l, m, k) in enumerate(g.labels):
        assert np.allclose(v[:, i], R0 * y00 * np.cos(k * a), rtol=0, atol=1e-14)


def test_feature_phi_invariances_and_gradient():
    g = group_o3_features(2, 2, 2, 5)
    K = all_invariant_tuples(g, 3, 5)
    c = np.random.default_rng(4).standard_normal(len(K))
    off = np.array([0, 5, 11], np.int32)
    pos = shell_positions(11, 5)
    phi, grad = oc.grad_naive(g.labels, K, c, off, pos, 5.0)
    assert grad.shape == (11, 3)
    # rotation about z of the positions (features unchanged)
    a = 0.7
    Q = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    rot = pos.copy()
    rot[:, :3] = pos[:, :3] @ Q.T
    assert np.allclose(oc.eval_naive(g.labels, K, c, off, rot, 5.0), phi, rtol=1e-12, atol=1e-12)
    # permuting (position, feature) pairs within an environment
    perm = np.concatenate([np.random.default_rng(6).permutation(5), 5 + np.random.default_rng(7).permutation(6)])
    assert np.allclose(oc.eval_naive(g.labels, K, c, off, pos[perm], 5.0), phi, rtol=1e-12, atol=1e-12)
    # the feature changes phi
    mu2 = pos.copy()
    mu2[:, 3] = -mu2[:, 3]
    assert not np.allclose(oc.eval_naive(g.labels, K, c, off, mu2, 5.0), phi)
    # gradient: central differences in the positions only
    h = 1e-6
    for j in (0, 7):
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[j, d] += h
            pm[j, d] -= h
            e = 0 if j < 5 else 1
            fd = (oc.eval_naive(g.labels, K, c, off, pp, 5.0)[e].real
                  - oc.eval_naive(g.labels, K, c, off, pm, 5.0)[e].real) / (2 * h)
            assert abs(grad[j, d] - fd) <= 1e-6 * max(1.0, abs(fd))
