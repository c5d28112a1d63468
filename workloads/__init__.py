"""Seeded synthetic workloads (inputs only; no evaluation arithmetic).

Both the oracle-based tests and the GPU path draw their inputs from here, so
this module holds nothing of the method itself: it fixes the basis sizes of
each workload and draws neighbour counts, relative positions and expansion
coefficients from numpy's PCG64 generator.

Recipe (the paper runs no evaluation experiment and ships no data; these
stand in for "atomic environments"):
  * positions: direction = normalised N(0, I_3) draw; radius uniform in the
    volume of the shell r_min < |r| < r_max, r = (r_min^3 + U (r_max^3 -
    r_min^3))^(1/3);
  * neighbour counts per workload (fixed, clipped Poisson, log-uniform);
  * coefficients c_k = N(0, 1) / (1 + deg_k)^q with deg_k = sum_t (n_t + l_t)
    supplied by the caller from its own listing of K;
  * seed = 1000 * workload id + stream (0 counts, 1 positions,
    2 coefficients, 3 species features).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

R_MIN, R_MAX = 0.5, 5.0


@dataclass(frozen=True)
class Workload:
    wid: int
    name: str
    n_env: int
    counts: str        # "fixed", "poisson", "loguniform"
    count_param: float
    count_lo: int
    count_hi: int
    nu_max: int
    degree_max: int
    n_max: int
    l_max: int
    coeff_power: int
    r_cut: float = 5.0
    group: int = 0          # 0 O(3) (shell in 3D), 1 torus (unit circle), 2 SO(2) (annulus)
    k_max: int = 0          # O(3) invariant feature degree (Sec. 5.4); positions get a mu column

    def spec(self) -> dict:
        return dict(nu_max=self.nu_max, degree_max=self.degree_max, n_max=self.n_max,
                    l_max=self.l_max, r_cut=self.r_cut, group=self.group, k_max=self.k_max)


WORKLOADS = {
    1: Workload(1, "forward-16x8", 16, "fixed", 8, 8, 8, 3, 8, 4, 4, 1),
    2: Workload(2, "forward-batch-4096", 4096, "poisson", 24.0, 4, 64, 4, 12, 6, 6, 2),
    3: Workload(3, "phi+forces-4096", 4096, "poisson", 24.0, 4, 64, 4, 12, 6, 6, 2),
    4: Workload(4, "uneven-32768", 32768, "loguniform", 0.0, 2, 96, 5, 14, 8, 8, 2),
    5: Workload(5, "large-basis-8192", 8192, "poisson", 40.0, 1, 128, 6, 16, 10, 10, 2),
    # planar groups (Sec. 2.2, 2.3): for SO(2) l_max is the largest |m|
    6: Workload(6, "so2-4096", 4096, "poisson", 24.0, 4, 64, 6, 16, 8, 8, 2, group=2),
    7: Workload(7, "torus-4096", 4096, "poisson", 24.0, 4, 64, 8, 24, 0, 0, 2, group=1),
    # one invariant feature per neighbour (four species, mu in {-1, -1/3, 1/3, 1})
    8: Workload(8, "species-4096", 4096, "poisson", 24.0, 4, 64, 4, 12, 6, 6, 2, k_max=3),
}


def _rng(wid: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * wid + stream))


def neighbour_counts(w: Workload, n_env: int | None = None) -> np.ndarray:
    """Neighbour count of every environment (int64)."""
    E = w.n_env if n_env is None else n_env
    g = _rng(w.wid, 0)
    if w.counts == "fixed":
        J = np.full(E, int(w.count_param), dtype=np.int64)
    elif w.counts == "poisson":
        J = g.poisson(w.count_param, size=E).astype(np.int64)
    elif w.counts == "loguniform":
        u = g.uniform(np.log(w.count_lo), np.log(w.count_hi + 1), size=E)
        J = np.floor(np.exp(u)).astype(np.int64)
    else:
        raise ValueError(w.counts)
    return np.clip(J, w.count_lo, w.count_hi)


def positions(n: int, seed_wid: int) -> np.ndarray:
    """n relative positions uniform in the volume of the shell; [n, 3] float64."""
    g = _rng(seed_wid, 1)
    d = g.standard_normal((n, 3))
    d /= np.sqrt(np.sum(d * d, axis=1))[:, None]
    u = g.uniform(0.0, 1.0, size=n)
    r = (R_MIN ** 3 + u * (R_MAX ** 3 - R_MIN ** 3)) ** (1.0 / 3.0)
    return d * r[:, None]


def planar_positions(n: int, seed_wid: int, circle: bool) -> np.ndarray:
    """n positions in the plane z = 0: on the unit circle (torus) or uniform in
    the area of the annulus r_min < r < r_max (SO(2)); [n, 3] float64."""
    g = _rng(seed_wid, 1)
    th = g.uniform(-np.pi, np.pi, size=n)
    if circle:
        r = np.ones(n)
    else:
        u = g.uniform(0.0, 1.0, size=n)
        r = np.sqrt(R_MIN ** 2 + u * (R_MAX ** 2 - R_MIN ** 2))
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n)], axis=-1)


def batch(w: Workload, n_env: int | None = None):
    """(offsets int32 [E+1], positions float64 [N, 3]) for workload w."""
    J = neighbour_counts(w, n_env)
    offsets = np.zeros(len(J) + 1, dtype=np.int64)
    np.cumsum(J, out=offsets[1:])
    if w.group == 0:
        pos = positions(int(offsets[-1]), w.wid)
        if w.k_max > 0:
            pos = np.concatenate([pos, species_feature(int(offsets[-1]), w.wid)[:, None]], axis=1)
    else:
        pos = planar_positions(int(offsets[-1]), w.wid, circle=w.group == 1)
    return offsets.astype(np.int32), pos


def species_feature(n: int, seed_wid: int, n_species: int = 4) -> np.ndarray:
    """A species label per neighbour, encoded as mu = -1 + 2 s / (n_species - 1)."""
    g = _rng(seed_wid, 3)
    s = g.integers(0, n_species, size=n)
    return -1.0 + 2.0 * s / (n_species - 1)


def coefficients(w: Workload, degrees: np.ndarray) -> np.ndarray:
    """c_k = N(0,1) / (1 + deg_k)^q, one per tuple of K in canonical order."""
    g = _rng(w.wid, 2)
    z = g.standard_normal(len(degrees))
    return z / (1.0 + np.asarray(degrees, dtype=np.float64)) ** w.coeff_power


def subset(offsets: np.ndarray, n: int, seed: int = 7) -> np.ndarray:
    """Sorted indices of n environments: the smallest and the largest
    neighbour count plus a seeded uniform sample of the rest."""
    J = np.diff(np.asarray(offsets, dtype=np.int64))
    E = len(J)
    if n >= E:
        return np.arange(E)
    pick = {int(np.argmin(J)), int(np.argmax(J))}
    g = np.random.Generator(np.random.PCG64(seed))
    rest = g.permutation(E)
    for e in rest:
        if len(pick) >= n:
            break
        pick.add(int(e))
    return np.array(sorted(pick), dtype=np.int64)


def gather(offsets: np.ndarray, pos: np.ndarray, envs: np.ndarray):
    """CSR batch restricted to the environments `envs` (in that order)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    parts, counts = [], []
    for e in envs:
        a, b = offsets[e], offsets[e + 1]
        parts.append(pos[a:b])
        counts.append(b - a)
    new_off = np.zeros(len(envs) + 1, dtype=np.int64)
    np.cumsum(counts, out=new_off[1:])
    p = np.concatenate(parts, axis=0) if parts else np.zeros((0, 3))
    return new_off.astype(np.int32), p


def random_A(n_env: int, P1: int, seed: int) -> np.ndarray:
    """Complex one-particle values with i.i.d. N(0,1) parts, for tests of the
    contraction alone; [n_env, P1] complex128."""
    g = np.random.Generator(np.random.PCG64(seed))
    return g.standard_normal((n_env, P1)) + 1j * g.standard_normal((n_env, P1))


def random_A_conj(n_env: int, labels, seed: int) -> np.ndarray:
    """Random one-particle values with the symmetry of pooled complex spherical
    harmonics, A[n, l, -m] = (-1)^m conj(A[n, l, m]) (so A[n, l, 0] is real);
    labels: the (n, l, m) of each one-particle index.  [n_env, P1] complex128."""
    A = random_A(n_env, len(labels), seed)
    where = {tuple(int(v) for v in t): i for i, t in enumerate(labels)}
    for i, (n, l, m) in enumerate(labels):
        n, l, m = int(n), int(l), int(m)
        if m == 0:
            A[:, i] = A[:, i].real
        elif m < 0:
            A[:, i] = (-1) ** m * np.conj(A[:, where[(n, l, -m)]])
    return A
