"""Pins of the oracle's index sets against independent counts and the paper.

Oracle functions pinned: onebody_o3, onebody_torus, invariant_tuples,
all_invariant_tuples, partitions_exact(_public), torus_aux_count_theorem.
"""

import itertools
import math

import pytest

from oracle import indexsets as ix


# ---- one-particle lists --------------------------------------------------------
@pytest.mark.parametrize("nmax,lmax,D,expect", [(4, 4, 8, 125), (6, 6, 12, 343), (8, 8, 14, 680),
                                                 (10, 10, 16, 1141)])
def test_onebody_counts(nmax, lmax, D, expect):
    # sum over (n, l) with n + l <= D of (2l + 1), counted directly
    direct = sum(2 * l + 1 for n in range(nmax + 1) for l in range(lmax + 1) if n + l <= D)
    assert direct == expect
    assert len(ix.onebody_o3(nmax, lmax, D)) == expect


def test_onebody_order_is_canonical():
    lab = ix.onebody_o3(3, 3, 4)
    keys = [(n + l, l, m) for (n, l, m) in lab]
    assert keys == sorted(keys)
    assert len(set(lab)) == len(lab)
    assert all(abs(m) <= l for (_, l, m) in lab)  # Sec. 2.4: |m| <= l
    assert ix.onebody_torus(3) == [0, -1, 1, -2, 2, -3, 3]


# ---- K against brute force and an independent multiset count ------------------
def brute_force_K(group, nu, D):
    out = []
    for t in itertools.combinations_with_replacement(range(len(group)), nu):
        if group.is_invariant(t) and group.degree(t) <= D:
            out.append(t)
    return out


@pytest.mark.parametrize("nu", [1, 2, 3])
def test_K_matches_brute_force_o3(nu):
    g = ix.group_o3(2, 2, 4)
    assert ix.invariant_tuples(g, nu, 4) == brute_force_K(g, nu, 4)


@pytest.mark.parametrize("nu,D", [(2, 6), (3, 6), (4, 5)])
def test_K_matches_brute_force_torus(nu, D):
    g = ix.group_torus(D)
    assert ix.invariant_tuples(g, nu, D) == brute_force_K(g, nu, D)


def multiset_count(nmax, lmax, D, nu):
    """#K_O3(nu, D) by a dynamic program over one-particle *types* with
    multiplicities (no tuple is ever listed): state (size, m-sum, l-parity,
    degree)."""
    types = [(n, l, m) for n in range(nmax + 1) for l in range(lmax + 1) if n + l <= D
             for m in range(-l, l + 1)]
    dp = {(0, 0, 0, 0): 1}
    for (n, l, m) in types:
        new = dict(dp)
        for (s, ms, lp, dg), cnt in dp.items():
            mult = 1
            while s + mult <= nu and dg + mult * (n + l) <= D:
                key = (s + mult, ms + mult * m, (lp + mult * l) % 2, dg + mult * (n + l))
                new[key] = new.get(key, 0) + cnt
                mult += 1
        dp = new
    return sum(c for (s, ms, lp, dg), c in dp.items() if s == nu and ms == 0 and lp == 0)


@pytest.mark.parametrize("nmax,lmax,D,nu_max", [(4, 4, 8, 3), (6, 6, 12, 4), (3, 5, 7, 4)])
def test_K_counts_match_multiset_dp(nmax, lmax, D, nu_max):
    g = ix.group_o3(nmax, lmax, D)
    for nu in range(1, nu_max + 1):
        assert len(ix.invariant_tuples(g, nu, D)) == multiset_count(nmax, lmax, D, nu)


def test_K_properties():
    g = ix.group_o3(4, 4, 8)
    K = ix.all_invariant_tuples(g, 3, 8)
    assert len(K) == len(set(K))
    for k in K:
        assert list(k) == sorted(k)
        assert sum(g.m[i] for i in k) == 0          # Sec. 2.4 rotation constraint
        assert sum(g.l[i] for i in k) % 2 == 0      # inversion constraint
        assert sum(g.deg[i] for i in k) <= 8        # total degree, p = 1
    # nu = 1: exactly the (n, l even, m = 0) functions (sum over K starts at nu = 1)
    k1 = [k for k in K if len(k) == 1]
    assert sorted(g.labels[k[0]] for k in k1) == sorted(
        (n, l, 0) for n in range(5) for l in range(0, 5, 2) if n + l <= 8)


# ---- integer partitions (Sec. 5.1) ------------------------------------------------
def test_partition_textbook_values():
    # p(n) = sum_k pi(k, n): p(10) = 42, p(20) = 627, p(30) = 5604
    for n, p in [(10, 42), (20, 627), (30, 5604), (1, 1), (5, 7)]:
        assert sum(ix.partitions_exact_public(k, n) for k in range(1, n + 1)) == p
    # pi(2, n) = floor(n / 2); pi(n, n) = 1; pi(0, n) = 0 (paper's convention)
    for n in range(1, 30):
        assert ix.partitions_exact_public(2, n) == n // 2
        assert ix.partitions_exact_public(n, n) == 1
        assert ix.partitions_exact_public(0, n) == 0


def test_partition_bounds_sec51():
    # (1/nu!) C(D-1, nu-1) <= pi(nu, D) <= (D + nu(nu-1)/2)^(nu-1) / (nu! (nu-1)!)
    for nu in range(1, 7):
        for D in range(nu, 40):
            p = ix.partitions_exact_public(nu, D)
            lo = math.comb(D - 1, nu - 1) / math.factorial(nu)
            hi = (D + nu * (nu - 1) / 2) ** (nu - 1) / (math.factorial(nu) * math.factorial(nu - 1))
            assert lo <= p <= hi + 1e-9


def test_partitions_by_brute_force():
    for nu in range(1, 5):
        for D in range(0, 13):
            cnt = sum(1 for t in itertools.combinations_with_replacement(range(1, D + 1), nu) if sum(t) == D)
            assert ix.partitions_exact_public(nu, D) == (cnt if nu > 0 else 0)


# ---- torus slices: exact formula of the slice lemma's proof (Sec. 5.2) -------------
def slice_count_enumerated(mu, D):
    """#E_T(mu, D): sorted nonzero m-tuples of length mu, sum 0, sum |m| = D."""
    vals = [m for m in range(-D, D + 1) if m != 0]
    return sum(1 for t in itertools.combinations_with_replacement(vals, mu)
               if sum(t) == 0 and sum(abs(m) for m in t) == D)


@pytest.mark.parametrize("mu", [2, 3, 4])
def test_torus_slice_formula(mu):
    for D in range(1, 13):
        if D % 2:
            assert slice_count_enumerated(mu, D) == 0   # property (2)
            continue
        formula = sum(ix.partitions_exact_public(k, D // 2) * ix.partitions_exact_public(mu - k, D // 2)
                      for k in range(0, mu + 1))
        assert slice_count_enumerated(mu, D) == formula


def test_torus_K_difference_property3():
    # #K_T(nu, D) - #K_T(nu, D-1) = sum_{k=1}^{nu} #E_T(k, D)
    nu = 4
    for D in range(1, 10):
        a = len(ix.invariant_tuples(ix.group_torus(D), nu, D))
        b = len(ix.invariant_tuples(ix.group_torus(D - 1), nu, D - 1)) if D >= 1 else 0
        assert a - b == sum(slice_count_enumerated(k, D) for k in range(1, nu + 1))


# ---- p-norm degree sets (Sec. 2.5: p = 2 and p = infinity) ----------------------
def brute_force_K_p(group, nu, D, p):
    """Every multiset of one-particle indices, kept when invariant and its element
    degrees have p-norm <= D (floating-point norm, compared with a margin)."""
    out = []
    for t in itertools.combinations_with_replacement(range(len(group)), nu):
        d = [group.deg[i] for i in t]
        norm = max(d) if p == math.inf else sum(x ** p for x in d) ** (1.0 / p)
        if group.is_invariant(t) and norm <= D + 1e-9:
            out.append(t)
    return out


@pytest.mark.parametrize("p", [2, math.inf])
@pytest.mark.parametrize("nu", [1, 2, 3])
def test_K_p_matches_brute_force_o3(nu, p):
    g = ix.group_o3(2, 2, 4)
    assert ix.invariant_tuples(g, nu, 4, p) == brute_force_K_p(g, nu, 4, p)


@pytest.mark.parametrize("p", [2, math.inf])
@pytest.mark.parametrize("nu,D", [(2, 5), (3, 4), (4, 3)])
def test_K_p_matches_brute_force_torus(nu, D, p):
    g = ix.group_torus(D)
    assert ix.invariant_tuples(g, nu, D, p) == brute_force_K_p(g, nu, D, p)


def test_K_p_nested_and_equal_for_single_elements():
    # ||k||_inf <= ||k||_2 <= ||k||_1, so K^1 within K^2 within K^inf; one element: all equal
    g = ix.group_o3(3, 3, 6)
    for nu in (1, 2, 3, 4):
        k1, k2, ki = (set(ix.invariant_tuples(g, nu, 6, p)) for p in (1, 2, math.inf))
        assert k1 <= k2 <= ki
        if nu == 1:
            assert k1 == k2 == ki
        else:
            assert len(k1) < len(k2) < len(ki)


@pytest.mark.parametrize("D", [3, 4, 7, 10])
def test_K_p_torus_pairs_closed_form(D):
    # torus, nu = 2: the invariant pairs are {m, -m}, m >= 0, with degree vector (m, m):
    # p = 1: 2m <= D;  p = 2: 2 m^2 <= D^2;  p = inf: m <= D
    g = ix.group_torus(D)
    assert len(ix.invariant_tuples(g, 2, D, 1)) == D // 2 + 1
    assert len(ix.invariant_tuples(g, 2, D, 2)) == math.isqrt(D * D // 2) + 1
    assert len(ix.invariant_tuples(g, 2, D, math.inf)) == D + 1
