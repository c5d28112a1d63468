"""Index sets of the oracle: one-particle lists, invariant tuples, partitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed:
  * O(3) one-particle index k = (n, l, m), |m| <= l  (Sec. 2.4)
  * invariant tuples: sum of m equal to 0, sum of l even  (Sec. 2.4)
  * torus one-particle index m, invariant tuples sum m = 0  (Sec. 2.3)
  * SO(2) one-particle index (n, m), invariant tuples sum m = 0; degree
    n + |m|  (Sec. 2.2, Sec. 2.5)
  * O(3) with an invariant feature, index (n, l, m, k), degree n + l + k
    (Sec. 5.4)
  * total degree p = 1: sum over the tuple of (n_t + l_t), resp. |m_t|
    (Sec. 2.5, Eq. (2.3); Sec. 3 explicit sets K_G(nu, D)); the other
    degree notions of Sec. 2.5, the p-norm of the per-element degrees, for
    p = 2 and p = infinity (the maximal element degree)
  * integer partitions pi(k, n) of n into exactly k positive parts (Sec. 5.1)

Canonical order (the paper leaves it open; fixed reading):
  * O(3): one-particle triples sorted by (n + l, l, m) ascending.
  * torus: m sorted by (|m|, m) ascending, i.e. 0, -1, 1, -2, 2, ...
  * SO(2): pairs (n, m) sorted by (n + |m|, |m|, m) ascending.
  * O(3) with a feature: (n, l, m, k) sorted by (n + l + k, l, k, m).
  A tuple is the non-decreasing list of positions in that list; sets of
  tuples are ordered by length, then lexicographically.  The element of
  largest degree is therefore the last one.
"""

from __future__ import annotations

import math
from functools import lru_cache


# --------------------------------------------------------------------------
# one-particle lists
# --------------------------------------------------------------------------

def onebody_o3(n_max: int, l_max: int, degree_max: int) -> list[tuple[int, int, int]]:
    """All (n, l, m) with 0<=n<=n_max, 0<=l<=l_max, |m|<=l, n+l<=D.

    Sec. 2.4 (phi_nlm = R_n Y_l^m, |m| <= l) with the degree n + l of
    Sec. 2.5; n starts at 0 (R_0 = T_0 = 1).  Canonical order (n+l, l, m).
    """
    out = []
    for n in range(n_max + 1):
        for l in range(l_max + 1):
            if n + l > degree_max:
                continue
            for m in range(-l, l + 1):
                out.append((n, l, m))
    out.sort(key=lambda t: (t[0] + t[1], t[1], t[2]))
    return out


def onebody_o3_features(n_max: int, l_max: int, k_max: int, degree_max: int) -> list[tuple[int, int, int, int]]:
    """O(3) with one invariant feature (Sec. 5.4): phi_nlmk = R_n Y_l^m T_k(mu),
    degree n + l + k <= D; quadruples (n, l, m, k) sorted by (n + l + k, l, k, m)
    (the k tie-break keeps the 2l+1 functions of one (n, l, k) consecutive;
    with k_max = 0 this is the plain O(3) order)."""
    out = [(n, l, m, k) for n in range(n_max + 1) for l in range(l_max + 1) for k in range(k_max + 1)
           if n + l + k <= degree_max for m in range(-l, l + 1)]
    out.sort(key=lambda t: (t[0] + t[1] + t[3], t[1], t[3], t[2]))
    return out


def onebody_so2(n_max: int, m_max: int, degree_max: int) -> list[tuple[int, int]]:
    """SO(2) one-particle pairs (n, m), Sec. 2.2 (phi_nm = R_n(r) e^{-i theta m}),
    n <= n_max, |m| <= m_max, degree n + |m| <= D, sorted by (n + |m|, |m|, m)."""
    out = [(n, m) for n in range(n_max + 1) for m in range(-m_max, m_max + 1) if n + abs(m) <= degree_max]
    out.sort(key=lambda t: (t[0] + abs(t[1]), abs(t[1]), t[1]))
    return out


def onebody_torus(degree_max: int) -> list[int]:
    """All m with |m| <= D (Sec. 2.3, phi_m = e^{i theta m}); order (|m|, m)."""
    out = list(range(-degree_max, degree_max + 1))
    out.sort(key=lambda m: (abs(m), m))
    return out


# --------------------------------------------------------------------------
# the group-specific data used by enumeration and by the graph builders
# --------------------------------------------------------------------------

class Group:
    """Per-one-particle quantities a group needs: degree, m, l parity.

    ``deg[i]``   degree of one-particle function i (n+l, resp. |m|)
    ``m[i]``     its m quantum number
    ``l[i]``     its l (0 for the torus)
    ``check_l``  whether the inversion constraint (sum l even) applies
    """

    def __init__(self, name, labels, deg, m, l, check_l):
        self.name = name
        self.labels = labels
        self.deg = deg
        self.m = m
        self.l = l
        self.check_l = check_l

    def __len__(self):
        return len(self.labels)

    def is_invariant(self, tup) -> bool:
        """Sec. 2.3 / 2.4: sum m_t = 0 and (O(3) only) sum l_t even."""
        if sum(self.m[i] for i in tup) != 0:
            return False
        if self.check_l and sum(self.l[i] for i in tup) % 2 != 0:
            return False
        return True

    def degree(self, tup) -> int:
        """Total degree, p = 1 (Sec. 2.5)."""
        return sum(self.deg[i] for i in tup)

    def within(self, tup, degree_max: int, p=1) -> bool:
        """||k||_p <= D for the element degrees (Sec. 2.5); p = 1, 2 or math.inf,
        compared in integers (sum of squares against D^2 for p = 2)."""
        d = [self.deg[i] for i in tup]
        if p == 1:
            return sum(d) <= degree_max
        if p == 2:
            return sum(x * x for x in d) <= degree_max * degree_max
        if p == math.inf:
            return max(d, default=0) <= degree_max
        raise ValueError(f"p must be 1, 2 or inf, got {p}")


def group_o3(n_max: int, l_max: int, degree_max: int) -> Group:
    lab = onebody_o3(n_max, l_max, degree_max)
    return Group("O3", lab, [n + l for (n, l, m) in lab], [m for (_, _, m) in lab],
                 [l for (_, l, _) in lab], True)


def group_o3_features(n_max: int, l_max: int, k_max: int, degree_max: int) -> Group:
    """Sec. 5.4: the invariance conditions of O(3) (sum m = 0, sum l even); the
    feature only adds to the degree."""
    lab = onebody_o3_features(n_max, l_max, k_max, degree_max)
    return Group("O3f", lab, [n + l + k for (n, l, m, k) in lab], [m for (_, _, m, _) in lab],
                 [l for (_, l, _, _) in lab], True)


def group_so2(n_max: int, m_max: int, degree_max: int) -> Group:
    """Sec. 2.2: invariance is sum m = 0 only (no parity constraint)."""
    lab = onebody_so2(n_max, m_max, degree_max)
    return Group("SO2", lab, [n + abs(m) for (n, m) in lab], [m for (_, m) in lab],
                 [abs(m) for (_, m) in lab], False)


def group_torus(degree_max: int) -> Group:
    lab = onebody_torus(degree_max)
    return Group("T", lab, [abs(m) for m in lab], list(lab), [0] * len(lab), False)


# --------------------------------------------------------------------------
# invariant tuple sets K_G(nu, D)
# --------------------------------------------------------------------------

def invariant_tuples(group: Group, nu: int, degree_max: int, p=1) -> list[tuple[int, ...]]:
    """K_G^p(nu, D): non-decreasing index tuples of length nu, invariant, ||k||_p <= D.

    Sec. 3 (explicit sets K_T, K_SO(2), K_O(3)).  Plain depth-first listing
    in lexicographic order.  Two exact prunings, neither of which drops a
    member of K: the degree budget (the one-particle list is sorted by
    degree, so later elements cost at least deg[i] each), and the m-sum
    (every one-particle function has |m| <= l <= its degree, resp. |m| equal
    to its degree, so the remaining degree budget bounds how far sum m can
    still move).  Membership itself is decided by is_invariant.

    For p = 2 and p = infinity (Eq. (2.3)) the listing prunes only by the
    degree of the next element (no later element may exceed D, and for p = 2
    each costs at least deg[i]^2 of D^2) and by the m-sum (every later
    element has |m| <= D); membership is decided by within() and
    is_invariant.
    """
    P = len(group)
    deg = group.deg
    mm = group.m
    out: list[tuple[int, ...]] = []
    cur: list[int] = []
    if p != 1:
        D = degree_max

        def rec_p(start: int, left: int, sq: int, msum: int):
            if left == 0:
                t = tuple(cur)
                if group.within(t, D, p) and group.is_invariant(t):
                    out.append(t)
                return
            for i in range(start, P):
                if deg[i] > D or (p == 2 and sq + deg[i] * deg[i] * left > D * D):
                    break
                ms = msum + mm[i]
                if abs(ms) > (left - 1) * D:
                    continue
                cur.append(i)
                rec_p(i, left - 1, sq + deg[i] * deg[i], ms)
                cur.pop()

        rec_p(0, nu, 0, 0)
        return out

    def rec(start: int, left: int, budget: int, msum: int):
        if left == 0:
            t = tuple(cur)
            if group.is_invariant(t):
                out.append(t)
            return
        for i in range(start, P):
            # every later element has degree >= deg[i]
            if deg[i] * left > budget:
                break
            ms = msum + mm[i]
            if abs(ms) > budget - deg[i]:
                continue
            cur.append(i)
            rec(i, left - 1, budget - deg[i], ms)
            cur.pop()

    rec(0, nu, degree_max, 0)
    return out


def all_invariant_tuples(group: Group, nu_max: int, degree_max: int, p=1) -> list[tuple[int, ...]]:
    """K = union over nu = 1..nu_max of K_G^p(nu, D), by length then lex (Eq. (1.1))."""
    out = []
    for nu in range(1, nu_max + 1):
        out.extend(invariant_tuples(group, nu, degree_max, p))
    return out


# --------------------------------------------------------------------------
# integer partitions (Sec. 5.1)
# --------------------------------------------------------------------------

@lru_cache(maxsize=None)
def partitions_exact(k: int, n: int) -> int:
    """pi(k, n): number of partitions of n into exactly k positive parts.

    Sec. 5.1 definition, with pi(0, n) = 0 as the paper sets it (and
    pi(0, 0) = 1 only as the base of the recursion below).  Recursion:
    either some part equals 1 (remove it: pi(k-1, n-1)) or all parts are
    >= 2 (subtract 1 from each: pi(k, n-k)).
    """
    if k == 0:
        return 1 if n == 0 else 0
    if n < k or k < 0:
        return 0
    return partitions_exact(k - 1, n - 1) + partitions_exact(k, n - k)


def partitions_exact_public(k: int, n: int) -> int:
    """pi(k, n) with the paper's convention pi(0, n) = 0 for every n."""
    if k == 0:
        return 0
    return partitions_exact(k, n)


def torus_aux_count_theorem(nu: int, degree_max: int) -> int:
    """Thm 3.2(ii): #A_T(nu, D) = 2 sum_{k=2}^{nu-1} sum_{n=1}^{floor(D/2)} pi(k, n)."""
    s = 0
    for k in range(2, nu):
        for n in range(1, degree_max // 2 + 1):
            s += partitions_exact_public(k, n)
    return 2 * s
