"""Computational DAG by the paper's node-insertion heuristics.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Sec. 2.6 (decomposition k = [k1, k2] <=> A_k = A_k1 * A_k2, auxiliary
nodes with zero coefficient, the graph G whose nodes of order >= 2 have
exactly two parents, insertion by increasing correlation order),
Algorithm 1 (Sec. 3.2) and Algorithm 2 (Sec. 3.3).

Readings fixed where the paper is silent (listed in the design doc):
  * G starts with every one-particle node [k], ids 0..P-1 in canonical order.
  * Tuples of K are inserted by length, then lexicographically.
  * "for all decompositions" is searched with the smaller part's size s
    running from floor(nu/2) down to 1; for each s the positions are taken
    in lexicographic (itertools.combinations) order, skipping a
    sub-multiset already tried.  The first split whose two parts are both
    in G is used, with parents (sub-multiset, complement).
  * The maximal-degree one-particle factor of Algorithm 1 is the last
    element of the sorted tuple (ties resolve to the last); Algorithm 2
    splits off the last min(n, nu - 1) elements, which is a maximal-norm
    sub-tuple for p = 1.
  * After the split-off part is inserted, the node itself is inserted by
    re-running the same search (the algorithm's final recursive call).
  * Node ids are insertion order; a recursively required node receives
    its id before the node that needed it.
"""

from __future__ import annotations

import itertools

from .indexsets import Group, all_invariant_tuples


class OracleGraph:
    """The DAG as plain Python lists.

    node_tuple[v]  sorted tuple of one-particle positions of node v
    parents[v]     (a, b) node ids, or None for one-particle nodes
    k_to_node[i]   node id of the i-th tuple of K (canonical order)
    K              the invariant tuples, canonical order
    """

    def __init__(self, group: Group, nu_max: int, degree_max: int,
                 algorithm: int = 1, alg_n: int = 1, p=1):
        self.group = group
        self.nu_max = nu_max
        self.degree_max = degree_max
        self.node_tuple: list[tuple[int, ...]] = []
        self.parents: list[tuple[int, int] | None] = []
        self.index: dict[tuple[int, ...], int] = {}
        # Sec. 2.6: first insert the one-particle nodes {[k]}
        for i in range(len(group)):
            self._add((i,), None)
        self.K = all_invariant_tuples(group, nu_max, degree_max, p)
        for k in self.K:
            if algorithm == 1:
                self.insert_alg1(k)
            else:
                self.insert_alg2(k, alg_n)
        self.k_to_node = [self.index[k] for k in self.K]

    # -- primitive --------------------------------------------------------
    def _add(self, tup, par):
        self.index[tup] = len(self.node_tuple)
        self.node_tuple.append(tup)
        self.parents.append(par)

    def _try_split(self, k) -> bool:
        """The 'for all decompositions' loop of Algorithms 1 and 2."""
        nu = len(k)
        for s in range(nu // 2, 0, -1):
            seen = set()
            for pos in itertools.combinations(range(nu), s):
                k1 = tuple(k[p] for p in pos)
                if k1 in seen:
                    continue
                seen.add(k1)
                rest = list(k)
                for p in reversed(pos):
                    del rest[p]
                k2 = tuple(rest)
                if k1 in self.index and k2 in self.index:
                    self._add(k, (self.index[k1], self.index[k2]))
                    return True
        return False

    # -- Algorithm 1 (Sec. 3.2) ---------------------------------------------
    def insert_alg1(self, k):
        if k in self.index:
            return
        if self._try_split(k):
            return
        # split off the one-particle factor of maximal degree (the last one);
        # [k^1] is always in G, so insert the remainder and retry.
        rest = k[:-1]
        self.insert_alg1(rest)
        self.insert_alg1(k)

    # -- Algorithm 2 (Sec. 3.3) ---------------------------------------------
    def insert_alg2(self, k, n):
        if k in self.index:
            return
        if self._try_split(k):
            return
        s = min(n, len(k) - 1)
        head = k[len(k) - s:]          # maximal-degree sub-tuple of length s
        rest = k[:len(k) - s]
        self.insert_alg1(head)         # this part is inserted with Algorithm 1
        self.insert_alg2(rest, n)
        self.insert_alg2(k, n)

    # -- derived statistics -------------------------------------------------
    def n_nodes(self) -> int:
        return len(self.node_tuple)

    def is_aux(self, v) -> bool:
        """Sec. 2.6: auxiliary = product node that is not invariant."""
        t = self.node_tuple[v]
        return len(t) >= 2 and not self.group.is_invariant(t)

    def aux_count(self) -> int:
        return sum(1 for v in range(self.n_nodes()) if self.is_aux(v))

    def layers(self) -> list[int]:
        """Layer of each node: leaves 0, otherwise 1 + max of the parents'."""
        lay = [0] * self.n_nodes()
        for v, p in enumerate(self.parents):
            if p is not None:
                lay[v] = 1 + max(lay[p[0]], lay[p[1]])
        return lay

    def child_counts(self) -> list[int]:
        cnt = [0] * self.n_nodes()
        for p in self.parents:
            if p is not None:
                cnt[p[0]] += 1
                cnt[p[1]] += 1
        return cnt
