"""Autotuner for the evaluation schedule of a graph.

The DAG (node list) is fixed by the insertion heuristic; how its evaluation
is laid out on the GPU is not: which kernel runs it (forest or remat), how
many pair-row entries, tree children or terms a lane takes per item, how
many hot slots get register accumulators, whether lanes and columns are
ordered by LDS bank group, the block size of the DAG kernel and how many
environments a block evaluates together.  tune()
searches these by coordinate descent for every available kernel, timing the
fused forward + reverse DAG launch (ace_contract with an adjoint) on the
caller's one-particle values, applies the fastest schedule to the graph and
records it in a JSON cache keyed by GPU architecture, basis and batch size
(ACE_AUTOTUNE_CACHE, default ~/.cache/ace_autotune.json).
Schedules tuned for the standard workloads ship with the package
(tuned.json) and are used when the user cache has no entry.
"""

from __future__ import annotations

import json
import os
import sys

from . import Graph, contract

# options that matter for each kernel, with the values searched
SPACE = {
    "forest": {
        "row_chunk": [16, 32, 64],
        "tree_chunk": [4, 8, 16, 32],
        "hot_columns": [0, 2, 4],
        "bank_schedule": [0, 1],
        "block_threads": [256, 512],
        "env_per_block": [1, 2],
    },
    "remat": {
        # searched jointly: two environments per block pay off only with the
        # 1024-thread blocks whose register bound keeps 16 waves per CU
        ("env_per_block", "block_threads"): [(1, 256), (1, 512), (1, 1024), (2, 512), (2, 1024)],
        "term_chunk": [16, 32, 64, 128, 256],
        "pair_slots": [-1, 0, 512, 1024, 2048],
        "hot_columns": [0, 2, 4],
    },
}


def cache_path() -> str:
    return os.environ.get("ACE_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                               "ace_autotune.json"))


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def _key(graph: Graph, n_env: int, device_name: str) -> str:
    s = graph.spec
    p = "" if s.get("degree_p", 1) == 1 else f"|p{s['degree_p']}"
    p += "" if not s.get("k_max", 0) else f"|k{s['k_max']}"
    return (f"{device_name}|g{s['group']}|nu{s['nu_max']}|D{s['degree_max']}|n{s['n_max']}|l{s['l_max']}"
            f"|alg{s['algorithm']}.{s['alg_n']}{p}|E{n_env}")


def _load(path: str | None = None) -> dict:
    try:
        with open(path or cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(data: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _time(graph: Graph, coeffs, A, reps: int) -> float:
    # A comes from ace_basis, so the launch folds conjugate pairs as ace_eval_grad does
    import torch
    for _ in range(2):
        contract(graph, coeffs, A, with_grad=True, conj_symmetric=True)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        contract(graph, coeffs, A, with_grad=True, conj_symmetric=True)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def arch(device) -> str:
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def _available(graph: Graph, kind: str) -> bool:
    from . import AceError
    cur = graph.get_schedule()
    try:
        graph.set_schedule(schedule=kind)
        return graph.schedule_kind() == kind
    except AceError:
        return False
    finally:
        graph.set_schedule(**cur)


def tune(graph: Graph, coeffs, A, *, reps: int = 5, use_cache: bool = True, verbose: bool = False,
         kinds=None) -> dict:
    """Pick and apply the fastest schedule for this graph and batch (A: [E, P1, 2],
    one-particle values from ace_basis).

    kinds: kernels to consider (default: every one the graph supports).
    Returns {"opts": ..., "ms": ..., "tried": [(opts, ms), ...], "cached": bool}.
    """
    dev = A.device
    key = _key(graph, A.shape[0], arch(dev))
    if use_cache:
        for data in (_load(), _load(SHIPPED)):
            if key in data and (kinds is None or data[key]["opts"].get("schedule") in kinds):
                opts = data[key]["opts"]
                graph.set_schedule(**opts)
                return {"opts": opts, "ms": data[key]["ms"], "tried": [], "cached": True}
    kinds = [k for k in (kinds or SPACE) if k in SPACE and _available(graph, k)]
    if not kinds:
        return {"opts": graph.get_schedule(), "ms": None, "tried": [], "cached": False}
    tried = []
    best, best_ms = None, float("inf")
    for kind in kinds:
        start = dict(graph.get_schedule(), schedule=kind)
        graph.set_schedule(**start)
        kbest, kms = start, _time(graph, coeffs, A, reps)
        tried.append((dict(kbest), kms))
        for name_, values in SPACE[kind].items():
            names = name_ if isinstance(name_, tuple) else (name_,)
            for v in values:
                vals = v if isinstance(name_, tuple) else (v,)
                if all(kbest[n] == x for n, x in zip(names, vals)):
                    continue
                cand = dict(kbest)
                cand.update(zip(names, vals))
                graph.set_schedule(**cand)
                ms = _time(graph, coeffs, A, reps)
                tried.append((cand, ms))
                if verbose:
                    print(f"[autotune] {cand}: {ms:.4f} ms", file=sys.stderr, flush=True)
                if ms < kms:
                    kbest, kms = cand, ms
        if kms < best_ms:
            best, best_ms = kbest, kms
    graph.set_schedule(**best)
    if use_cache:
        data = _load()
        data[key] = {"opts": best, "ms": best_ms}
        _store(data)
    return {"opts": best, "ms": best_ms, "tried": tried, "cached": False}
