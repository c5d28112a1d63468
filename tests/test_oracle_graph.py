"""Pins of the oracle's DAG builder (Algorithms 1 and 2) against the paper.

Oracle functions pinned: OracleGraph (insert_alg1, insert_alg2, _try_split),
aux_count, layers.
"""

import math

import pytest

from oracle.indexsets import group_o3, group_torus, torus_aux_count_theorem
from oracle.graph import OracleGraph


# ---- Theorem 3.2(ii): exact auxiliary count of Algorithm 1 on the torus ----------
@pytest.mark.parametrize("nu", [3, 4, 5, 6])
@pytest.mark.parametrize("D", [2, 4, 6, 8, 10, 12, 16])
def test_theorem_3_2_ii_exact_torus_aux_count(nu, D):
    G = OracleGraph(group_torus(D), nu, D)
    assert G.aux_count() == torus_aux_count_theorem(nu, D)


def test_theorem_3_2_ii_spot_values():
    # 2 * sum_{k=2}^{3} sum_{n=1}^{4} pi(k, n) = 2 * ((0+1+1+2) + (0+0+1+1)) = 12
    assert torus_aux_count_theorem(4, 8) == 12
    assert OracleGraph(group_torus(8), 4, 8).aux_count() == 12


def test_torus_nu3_split_is_max_element_plus_pair():
    # proof of Thm 3.2(ii): an independent nu = 3 tuple [m1, -m2, -m3], m1 = m2 + m3,
    # is split as [m1] and the auxiliary pair [-m2, -m3]
    D = 8
    G = OracleGraph(group_torus(D), 3, D)
    lab = G.group.labels
    for v, t in enumerate(G.node_tuple):
        if len(t) != 3:
            continue
        a, b = G.parents[v]
        ta, tb = G.node_tuple[a], G.node_tuple[b]
        if G.is_aux(a) or G.is_aux(b):
            one, pair = (ta, tb) if len(ta) == 1 else (tb, ta)
            ms = [lab[i] for i in t]
            big = max(ms, key=abs)
            assert lab[one[0]] == big
            assert sorted(lab[i] for i in pair) == sorted(ms[:ms.index(big)] + ms[ms.index(big) + 1:])


# ---- worked examples of Sec. 2.6 and Sec. 5.2 --------------------------------------
def tor(G, ms):
    lab = G.group.labels
    return tuple(sorted(lab.index(m) for m in ms))


def invariant_splits(G, ms):
    """All splits of the m-tuple into two invariant, non-empty sub-multisets."""
    import itertools
    out = set()
    n = len(ms)
    for s in range(1, n // 2 + 1):
        for pos in itertools.combinations(range(n), s):
            a = tuple(sorted(ms[p] for p in pos))
            b = tuple(sorted(ms[p] for p in range(n) if p not in pos))
            if sum(a) == 0 and sum(b) == 0:
                out.add(tuple(sorted([a, b])))
    return out


def test_worked_examples_dependent_independent():
    D = 12
    G = OracleGraph(group_torus(D), 6, D)
    # [1, 0, -1] = [0] . [1, -1] is dependent
    assert invariant_splits(G, [1, 0, -1]) == {((-1, 1), (0,))}
    v = G.index[tor(G, [1, 0, -1])]
    a, b = G.parents[v]
    assert {G.node_tuple[a], G.node_tuple[b]} == {tor(G, [0]), tor(G, [1, -1])}
    # [1, 1, -2] is independent: only the auxiliary [1, 1] completes it
    assert invariant_splits(G, [1, 1, -2]) == set()
    v = G.index[tor(G, [1, 1, -2])]
    a, b = G.parents[v]
    assert {G.node_tuple[a], G.node_tuple[b]} == {tor(G, [-2]), tor(G, [1, 1])}
    assert G.is_aux(G.index[tor(G, [1, 1])])
    # [3, 2, 1, -1, -2, -3] has (at least) two distinct decompositions (Sec. 5.2)
    splits = invariant_splits(G, [3, 2, 1, -1, -2, -3])
    assert tuple(sorted([(-3, 3), (-2, -1, 1, 2)])) in splits
    assert tuple(sorted([(-2, 2), (-3, -1, 1, 3)])) in splits


# ---- structural invariants of the DAG (Sec. 2.6) ------------------------------------
@pytest.mark.parametrize("alg,n", [(1, 1), (2, 2)])
@pytest.mark.parametrize("spec", [(4, 4, 8, 3), (3, 3, 8, 4)])
def test_dag_structure_o3(spec, alg, n):
    nmax, lmax, D, nu = spec
    g = group_o3(nmax, lmax, D)
    G = OracleGraph(g, nu, D, alg, n)
    P = len(g)
    # one-particle nodes first, in canonical order
    assert G.node_tuple[:P] == [(i,) for i in range(P)]
    # every tuple of K is a node exactly once
    assert len(set(G.k_to_node)) == len(G.K)
    assert len(G.index) == G.n_nodes()
    ch = G.child_counts()
    for v in range(P, G.n_nodes()):
        a, b = G.parents[v]
        assert a < v and b < v                                    # parents precede
        assert tuple(sorted(G.node_tuple[a] + G.node_tuple[b])) == G.node_tuple[v]  # mset union
        inv = g.is_invariant(G.node_tuple[v])
        assert G.is_aux(v) == (not inv)                           # aux = non-invariant
        if ch[v] == 0:
            assert inv                                            # nothing wasted
    # non-invariant nodes are never tuples of K
    kset = set(G.K)
    for v in range(P, G.n_nodes()):
        assert (G.node_tuple[v] in kset) == (not G.is_aux(v))


def test_alg2_preasymptotics_p1_worse_than_alg1():
    # Sec. 3.4: for p = 1 the pre-asymptotic behaviour of Algorithm 2 is slightly worse
    for spec in [(4, 4, 8, 3), (6, 6, 12, 4)]:
        nmax, lmax, D, nu = spec
        a1 = OracleGraph(group_o3(nmax, lmax, D), nu, D, 1).aux_count()
        a2 = OracleGraph(group_o3(nmax, lmax, D), nu, D, 2, 2).aux_count()
        assert a2 > a1


def test_nu2_needs_no_aux():
    G = OracleGraph(group_o3(4, 4, 8), 2, 8)
    assert G.aux_count() == 0
    assert max(G.layers()) == 1


def _golden_rows():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_worked_examples.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        kind, tup, exp = [x.strip() for x in line.split("|")]
        rows.append((kind, tup, exp))
    return rows


def test_golden_paper_examples():
    D = 12
    G = OracleGraph(group_torus(D), 6, D)
    for kind, tup, exp in _golden_rows():
        if kind == "aux_count":
            nu, Dv = [int(x.split("=")[1]) for x in tup.split(",")]
            assert OracleGraph(group_torus(Dv), nu, Dv).aux_count() == int(exp)
            assert torus_aux_count_theorem(nu, Dv) == int(exp)
            continue
        ms = [int(x) for x in tup.split(",")]
        parts = [tuple(sorted(int(x) for x in p.split(","))) for p in exp.split(";")] if exp != "-" else []
        splits = invariant_splits(G, ms)
        if kind == "dependent":
            assert tuple(sorted(parts)) in splits
        elif kind == "independent":
            assert splits == set()
        elif kind == "aux_split":
            v = G.index[tor(G, ms)]
            a, b = G.parents[v]
            assert {G.node_tuple[a], G.node_tuple[b]} == {tor(G, list(p)) for p in parts}
        elif kind == "two_splits":
            assert tuple(sorted(parts[:2])) in splits and tuple(sorted(parts[2:])) in splits


@pytest.mark.parametrize("p", [2, math.inf])
def test_alg2_fewer_aux_than_alg1_for_p_above_1(p):
    # Sec. 3.4 (discussion of the O(3) computations): for p > 1 the generalized
    # heuristic with n = 2 inserts fewer auxiliary nodes than Algorithm 1
    for nu, D, nl in [(3, 6, 3), (4, 5, 3)]:
        g = group_o3(nl, nl, D)
        a1 = OracleGraph(g, nu, D, 1, p=p).aux_count()
        a2 = OracleGraph(g, nu, D, 2, 2, p=p).aux_count()
        assert a2 < a1


@pytest.mark.parametrize("p", [2, math.inf])
def test_dag_structure_p_norm(p):
    g = group_o3(3, 3, 6)
    for alg, n in [(1, 1), (2, 2)]:
        G = OracleGraph(g, 4, 6, alg, n, p=p)
        kset = set(G.K)
        for v, par in enumerate(G.parents):
            if par is None:
                continue
            a, b = par
            assert a < v and b < v
            assert tuple(sorted(G.node_tuple[a] + G.node_tuple[b])) == G.node_tuple[v]
        assert all(G.node_tuple[G.k_to_node[q]] == k for q, k in enumerate(G.K))
        assert len(kset) == len(G.K)


def _hand_worked_lists():
    """Sections of tests/golden/alg2_torus_nu4_D6.txt: {(alg, n): [(id, tuple, parents)]}."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "alg2_torus_nu4_D6.txt")
    out, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            alg, n = line.strip("[]").split()
            cur = out.setdefault((int(alg[3:]), int(n[2:])), [])
            continue
        v, tup, par = [x.strip() for x in line.split("|")]
        cur.append((int(v), tuple(int(x) for x in tup.split(",")), tuple(int(x) for x in par.split(","))))
    return out


@pytest.mark.parametrize("alg,n", [(1, 1), (2, 2), (2, 3)])
def test_algorithms_match_hand_worked_torus_graph(alg, n):
    """Algorithms 1 and 2 (Sec. 3.2, 3.3) against node lists derived by hand
    for the torus, nu <= 4, D = 6: every product node, its id (insertion
    order: the split-off part before the remainder) and its parents.  With
    n = 3 the split-off triple is inserted by Algorithm 1, not by
    Algorithm 2; with n = 2 the split-off pair precedes the remainder."""
    expected = _hand_worked_lists()[(alg, n)]
    G = OracleGraph(group_torus(6), 4, 6, alg, n)
    assert G.n_nodes() == 13 + len(expected)
    for v, tup, par in expected:
        assert G.node_tuple[v] == tup, v
        assert G.parents[v] == par, v
    assert G.aux_count() == (6 if alg == 1 else 8)
    if alg == 1:
        assert torus_aux_count_theorem(4, 6) == 6
