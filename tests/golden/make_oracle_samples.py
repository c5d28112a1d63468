"""Write the oracle's phi and gradients on seeded environment subsets of the
32768-environment (nu <= 5, D <= 14) and 8192-environment (nu <= 6, D <= 16)
workloads, for the full-size GPU parity tests (the oracle needs about two
seconds per environment of the larger basis, too slow to run inside them).

    python tests/golden/make_oracle_samples.py [--procs 8]

Calls only oracle/ and the seeded input generators.  Each file holds the
subset (smallest and largest neighbour counts included), a fingerprint of its
inputs (positions and coefficients) that the tests recompute, phi and the
gradients.
"""

from __future__ import annotations

import argparse
import hashlib
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle.contraction import grad_naive  # noqa: E402
from oracle.indexsets import all_invariant_tuples, group_o3  # noqa: E402

SAMPLES = {4: 64, 5: 64}
_W = {}


def path_for(wid: int) -> str:
    return os.path.join(HERE, f"oracle_samples_w{wid}.npz")


def fingerprint(pos_subset: np.ndarray, coeffs: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pos_subset, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(coeffs, dtype=np.float64).tobytes())
    return h.hexdigest()


def _run(job):
    off, pos = job
    w, g, K, c = _W["w"], _W["g"], _W["K"], _W["c"]
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return grad_naive(g.labels, K, c, off, pos, w.r_cut)


def make(wid: int, procs: int) -> None:
    w = wl.WORKLOADS[wid]
    g = group_o3(w.n_max, w.l_max, w.degree_max)
    K = all_invariant_tuples(g, w.nu_max, w.degree_max)
    c = wl.coefficients(w, np.array([g.degree(k) for k in K]))
    _W.update(w=w, g=g, K=K, c=c)
    off, pos = wl.batch(w)
    envs = wl.subset(off, SAMPLES[wid])
    jobs = [wl.gather(off, pos, [e]) for e in envs]
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_run, jobs, chunksize=1)
    phi = np.concatenate([r[0] for r in res])
    grad = np.concatenate([r[1] for r in res])
    so, sp_ = wl.gather(off, pos, envs)
    np.savez_compressed(path_for(wid), envs=envs, offsets=so, phi=phi, grad=grad,
                        fingerprint=np.array(fingerprint(sp_, c)))
    print(f"workload {wid}: {len(envs)} environments, {len(sp_)} neighbours -> {path_for(wid)}", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=min(8, len(os.sched_getaffinity(0))))
    ap.add_argument("--workloads", default="4,5")
    a = ap.parse_args()
    for wid in (int(x) for x in a.workloads.split(",")):
        make(wid, a.procs)
