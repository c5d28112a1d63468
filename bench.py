#!/usr/bin/env python3
"""Throughput of phi + forces by recursive DAG contraction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 5]

One step = one pass of the whole path over the batch (one-particle basis,
DAG forward with the coefficient contraction, reverse pass, dA/dr chain)
through ace_eval_grad, inputs resident in HBM.  The same pass with the naive
per-tuple kernel is timed beside it.  Prints one JSON line.

The CPU baseline is the FP64 oracle as it stands, on a bounded sample of
the same workload, in worker processes started before the GPU is touched.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

METRIC = "environments/s (phi+forces) DAG vs naive on 1 MI355X at FP64 rel err ≤1e-9"
FP64_PEAK_TFLOPS = 78.6   # MI355X vector FP64
HBM_PEAK_GBS = 8000.0


# ---------------------------------------------------------------------------
# algorithmic operation counts of the DAG kernel (forward + reverse pass)
# ---------------------------------------------------------------------------
def dag_flops_per_env(stats: dict) -> dict:
    """Algorithmic flops of one environment in the fused forward + reverse
    DAG launch, by the per-node figures of the scope table:

    forward = 6 S + 3 T + 2 |K|   (S product nodes with children: a complex
              product; T childless product nodes: the real part of a product;
              each tuple of K: a real coefficient times a real part)
    reverse = 16 S + 8 T          (adjoint pushes to both parents)

    The kernel does more than this (it also returns Im phi), so the achieved
    rate computed from it is a lower bound.
    """
    S = stats["n_stored"]
    T = stats["n_childless"]
    K = stats["n_k"]
    fwd = 6 * S + 3 * T + 2 * K
    adj = 16 * S + 8 * T
    return dict(forward=fwd, reverse=adj, total=fwd + adj)


def naive_flops_per_env(stats: dict) -> dict:
    """Algorithmic flops of one environment in the naive forward + reverse launch:
    every tuple's product from its factors, C = sum_k (nu_k - 1) complex
    products; forward 6 C + 2 |K|; reverse by suffix products and
    prefix x suffix (12 C) plus the nu_k adjoint accumulations (2 per factor)."""
    C = stats["naive_cmuls"]
    K = stats["n_k"]
    fwd = 6 * C + 2 * K
    adj = 12 * C + 2 * (C + K)
    return dict(forward=fwd, reverse=adj, total=fwd + adj)


def source_hash() -> str:
    """Hash of the kernel and schedule sources (ties counter profiles to them)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "ace.hip", "ace_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2202_04140_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_key(workload: int, schedule: dict) -> str:
    """What a counter profile was taken on: the kernel and schedule-builder
    sources, the schedule options and the workload (together they fix the
    code object and the uploaded schedule arrays)."""
    import hashlib
    h = hashlib.sha256()
    h.update(source_hash().encode())
    h.update(json.dumps(schedule, sort_keys=True).encode())
    h.update(str(workload).encode())
    return h.hexdigest()[:16]


def traffic_path(workload: int) -> str:
    return os.path.join(ROOT, "profiles", f"dag_kernel_traffic_w{workload}.json")


def counters_path(workload: int) -> str:
    return os.path.join(ROOT, "profiles", f"dag_kernel_counters_w{workload}.json")


def _profile(path: str, workload: int, schedule: dict):
    """A committed counter profile if it was taken on this workload, these
    sources and this schedule, else None."""
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    return d if d.get("key") == profile_key(workload, schedule) else None


def profiled_traffic(workload: int, schedule: dict):
    """HBM bytes per launch of the dominant kernel from the committed counter profile."""
    d = _profile(traffic_path(workload), workload, schedule)
    return None if d is None else d.get("bytes_per_launch")


# ---------------------------------------------------------------------------
# CPU baseline (oracle) -- runs before any GPU initialisation
# ---------------------------------------------------------------------------
# Worker processes at most: the host share of one GPU on the machines this
# runs on is 16 cores, whatever the affinity mask shows.
MAX_WORKERS = 16
_W = {}


def _oracle_setup(wid):
    """The oracle's own listing of K and the coefficients drawn from it."""
    from oracle.indexsets import all_invariant_tuples, group_o3, group_so2, group_torus
    w = wl.WORKLOADS[wid]
    if w.group == 0 and w.k_max > 0:
        from oracle.indexsets import group_o3_features
        g = group_o3_features(w.n_max, w.l_max, w.k_max, w.degree_max)
    elif w.group == 0:
        g = group_o3(w.n_max, w.l_max, w.degree_max)
    elif w.group == 2:
        g = group_so2(w.n_max, w.l_max, w.degree_max)
    else:
        g = group_torus(w.degree_max)
    K = all_invariant_tuples(g, w.nu_max, w.degree_max)
    c = wl.coefficients(w, np.array([g.degree(k) for k in K]))
    _W.update(w=w, g=g, K=K, c=c)


def _worker_init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _worker_run(args):
    off, pos = args
    from oracle.contraction import grad_naive
    w, g, K, c = _W["w"], _W["g"], _W["K"], _W["c"]
    return grad_naive(g.labels, K, c, off, pos, w.r_cut)


def default_cpu_sample(wid: int) -> int:
    """Whole batch for the small workloads, a 512-environment subset (smallest
    and largest neighbour count included) for the 32768- and 8192-environment ones."""
    return 512 if wl.WORKLOADS[wid].n_env > 4096 else wl.WORKLOADS[wid].n_env


def cpu_baseline(wid: int, off: np.ndarray, pos: np.ndarray, n_sample: int, chunk: int = 8,
                 one_core_envs: int = 4):
    """The oracle on a seeded subset of the batch, on every core of the
    affinity mask (at most MAX_WORKERS single-threaded processes), and on a
    few environments of it on one core."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    t0 = time.perf_counter()
    _oracle_setup(wid)                      # inherited by the forked workers
    t_setup = time.perf_counter() - t0
    envs = wl.subset(off, n_sample)
    affinity = len(os.sched_getaffinity(0))
    cores = max(1, min(affinity, MAX_WORKERS))
    jobs = [wl.gather(off, pos, envs[i:i + chunk]) for i in range(0, len(envs), chunk)]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores, initializer=_worker_init) as pool:
        t0 = time.perf_counter()
        res = pool.map(_worker_run, jobs, chunksize=1)
        dt = time.perf_counter() - t0
    phi = np.concatenate([r[0] for r in res])
    grad = np.concatenate([r[1] for r in res])
    # one core: the first few environments of the subset in this process
    n1 = min(one_core_envs, len(envs))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        _worker_run(wl.gather(off, pos, envs[:n1]))
        dt1 = time.perf_counter() - t0
    cpu = open("/proc/cpuinfo").read()
    model = next((ln.split(":", 1)[1].strip() for ln in cpu.splitlines() if ln.startswith("model name")), "?")
    return envs, phi, grad, dict(value=len(envs) / dt, unit="environments/s", cores=cores, kind="oracle",
                                 sample=f"{len(envs)} environments of the same workload (seeded subset with the "
                                        f"smallest and largest neighbour count), phi + forces, {dt:.1f} s wall on "
                                        f"{cores} single-threaded processes ({model}, {affinity} cores in the "
                                        f"affinity mask); K listed once beforehand in {t_setup:.1f} s",
                                 one_core={"value": n1 / dt1, "unit": "environments/s", "envs": n1,
                                           "seconds": dt1})


# ---------------------------------------------------------------------------
# HBM traffic of the dominant kernel from two rocprofv3 counter databases
# ---------------------------------------------------------------------------
def _per_dispatch(db_path: str, counter: str):
    import sqlite3
    cur = sqlite3.connect(db_path).cursor()
    rows = cur.execute("select dispatch_id, kernel_name, value from counters_collection where counter_name = ?",
                       (counter,)).fetchall()
    acc = {}
    for d, name, v in rows:
        k = (d, name)
        acc[k] = acc.get(k, 0.0) + float(v)
    return acc


def pmc_table(dbs) -> dict:
    """{kernel: {counter: mean value per dispatch, "dispatches": n}} over rocprofv3 counter databases."""
    import sqlite3
    out = {}
    for db in dbs:
        cur = sqlite3.connect(db).cursor()
        rows = cur.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection").fetchall()
        acc = {}
        for d, name, cname, v in rows:
            k = (name, cname)
            acc.setdefault(k, {}).setdefault(d, 0.0)
            acc[k][d] += float(v)
        for (name, cname), per in acc.items():
            e = out.setdefault(name, {})
            e[cname] = sum(per.values()) / len(per)
            e["dispatches"] = max(e.get("dispatches", 0), len(per))
    return out


def _dominant_dag_kernel(table: dict) -> str:
    names = [n for n in table if "forest_kernel<true" in n or "remat_kernel<true" in n]
    if not names:
        raise RuntimeError("no forward + reverse DAG dispatch in the counter databases")
    return max(names, key=lambda n: table[n]["dispatches"])


def summarize_counters(dbs, workload: int, schedule: dict, out_path: str) -> dict:
    """Mean per dispatch of every counter of the dominant DAG kernel (the forest
    or remat kernel with its adjoint) over rocprofv3 counter databases, with
    the quantities derived from them."""
    table = pmc_table(dbs)
    kernel = _dominant_dag_kernel(table)
    v = table[kernel]
    out = dict(workload=workload, key=profile_key(workload, schedule), schedule=schedule, kernel=kernel,
               counters=v)
    if "SQ_INSTS_VALU_FLOPS_FP64" in v:
        # the counter adds 1 per FP64 add/mul and 2 per FMA of a wave; x64 lanes
        out["fp64_flops_per_launch"] = 64.0 * v["SQ_INSTS_VALU_FLOPS_FP64"]
    if "GRBM_GUI_ACTIVE" in v and "SQ_ACTIVE_INST_VALU" in v:
        cyc = v["GRBM_GUI_ACTIVE"] / 8.0                        # per XCD
        out["cycles"] = cyc
        out["valu_busy"] = 4.0 * v["SQ_ACTIVE_INST_VALU"] / (1024.0 * cyc)   # quad-cycles over 1024 SIMDs
        out["lds_active"] = v["SQ_LDS_IDX_ACTIVE"] / (256.0 * cyc)
        out["lds_bank_conflict_share"] = v["SQ_LDS_BANK_CONFLICT"] / max(1.0, v["SQ_LDS_IDX_ACTIVE"])
        out["waves_per_cu"] = 4.0 * v["SQ_WAVE_CYCLES"] / max(1.0, v["SQ_BUSY_CU_CYCLES"])
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def summarize_pmc(fetch_db: str, write_db: str, copy_mib: int, workload: int, schedule: dict, out_path: str) -> dict:
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the fused forward +
    reverse DAG kernel (the forest or remat kernel with its adjoint, whichever
    the run dispatched most), scaled by what the same counters read for a
    plain device copy of copy_mib MiB (copy_mib read + copy_mib written)."""
    res = {}
    kernel = None
    for counter, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        acc = _per_dispatch(db, counter)
        copies = [v for (d, n), v in acc.items() if "copyBuffer" in n or "copy" in n.lower()]
        names = {}
        for (d, n), v in acc.items():
            if "forest_kernel<true" in n or "remat_kernel<true" in n:
                names.setdefault(n, []).append(v)
        if not copies or not names:
            raise RuntimeError(f"{counter}: no copy or DAG dispatch in {db}")
        kernel = kernel or max(names, key=lambda n: len(names[n]))
        dag = names[kernel]
        copy_kib = max(copies)
        scale = copy_mib * 1024.0 / copy_kib
        res[counter] = dict(copy_kib=copy_kib, scale=scale, kernel_kib_mean=sum(dag) / len(dag),
                            kernel_dispatches=len(dag))
    fetch_b = res["FETCH_SIZE"]["kernel_kib_mean"] * 1024 * res["FETCH_SIZE"]["scale"]
    write_b = res["WRITE_SIZE"]["kernel_kib_mean"] * 1024 * res["WRITE_SIZE"]["scale"]
    out = dict(workload=workload, key=profile_key(workload, schedule), schedule=schedule, kernel=kernel,
               copy_mib=copy_mib, fetch_bytes=fetch_b, write_bytes=write_b, bytes_per_launch=fetch_b + write_b,
               counters=res)
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    return out


# ---------------------------------------------------------------------------
def per_env_errors(phi, phi_ref, grad, grad_ref, offsets) -> dict:
    """Largest per-environment norm-wise relative errors: |phi_e - ref_e| / |ref_e|
    over the environments whose |ref_e| is at least 1e-6 of the RMS (the others
    are counted as flagged), and ||g_e - ref_e|| / ||ref_e|| over each
    environment's gradient rows."""
    phi, phi_ref = np.asarray(phi), np.asarray(phi_ref)
    mag = np.abs(phi_ref)
    rms = float(np.sqrt(np.mean(mag ** 2))) if len(mag) else 0.0
    ok = mag >= 1e-6 * rms
    e_phi = np.abs(phi - phi_ref)[ok] / mag[ok]
    off = np.asarray(offsets, dtype=np.int64)
    d2 = np.add.reduceat(np.sum((grad - grad_ref) ** 2, axis=1), off[:-1]) if len(grad) else np.zeros(0)
    r2 = np.add.reduceat(np.sum(grad_ref ** 2, axis=1), off[:-1]) if len(grad) else np.zeros(0)
    has = (np.diff(off) > 0) & (r2 > 0)
    e_g = np.sqrt(d2[has] / r2[has])
    return dict(phi_max=float(e_phi.max()) if len(e_phi) else 0.0, phi_flagged=int((~ok).sum()),
                grad_max=float(e_g.max()) if len(e_g) else 0.0)


def dag_kernel_ms(ace, torch, G, tc, A, timed, steps, warmup) -> float:
    """The dominant kernel alone: the fused forward + reverse DAG launch
    (ace_contract on the basis output, conjugate pairs folded as in
    ace_eval_grad), timed with events on the stream it is launched on."""
    dev = A.device
    E = A.shape[0]
    phi = torch.empty((E, 2), dtype=torch.float64, device=dev)
    Abar = torch.empty_like(A)
    ws = G.workspace(E, dev)
    lib = ace.lib()
    stream = torch.cuda.current_stream(dev)

    def launch():
        st = lib.ace_contract(G.handle, tc.data_ptr(), E, A.data_ptr(), phi.data_ptr(), Abar.data_ptr(),
                              ws.data_ptr(), ws.numel(), ace.FLAG_CONJ_SYMMETRIC, ace._stream(dev))
        if st != 0:
            raise RuntimeError(lib.ace_last_error().decode())

    with torch.cuda.stream(stream):
        ms, _ = timed(launch, steps, warmup)
    return ms


def naive_kernel_ms(ace, torch, G, tc, A, timed, steps, warmup) -> float:
    """The naive forward + reverse launch alone (ace_contract with ACE_FLAG_NAIVE,
    its coefficient gather included), timed with events on its stream."""
    dev = A.device
    E = A.shape[0]
    phi = torch.empty((E, 2), dtype=torch.float64, device=dev)
    Abar = torch.empty_like(A)
    ws = G.workspace(E, dev, ace.FLAG_NAIVE)
    lib = ace.lib()

    def launch():
        st = lib.ace_contract(G.handle, tc.data_ptr(), E, A.data_ptr(), phi.data_ptr(), Abar.data_ptr(),
                              ws.data_ptr(), ws.numel(), ace.FLAG_NAIVE, ace._stream(dev))
        if st != 0:
            raise RuntimeError(lib.ace_last_error().decode())

    with torch.cuda.stream(torch.cuda.current_stream(dev)):
        ms, _ = timed(launch, steps, warmup)
    return ms


def small_workload_figures(ace, torch, dev, timed, graphed, args) -> dict:
    """phi + forces on the 4096-environment nu <= 4 workload, beside the headline."""
    w = wl.WORKLOADS[3]
    off, pos = wl.batch(w)
    E = len(off) - 1
    G = ace.Graph(w.nu_max, w.degree_max, w.n_max, w.l_max, r_cut=w.r_cut)
    tc = torch.from_numpy(wl.coefficients(w, G.k_degrees())).to(dev)
    toff = torch.from_numpy(off).to(dev)
    tpos = torch.from_numpy(pos).to(dev)
    phi = torch.empty((E, 2), dtype=torch.float64, device=dev)
    grad = torch.empty((len(pos), 3), dtype=torch.float64, device=dev)
    A = ace.basis(G, toff, tpos)
    if not args.no_tune:
        from paper_2202_04140_amd import autotune
        autotune.tune(G, tc, A, use_cache=not args.retune)
    ms, _ = timed(graphed(lambda: ace.eval_grad(G, tc, toff, tpos, out=(phi, grad))), 20, 5)
    ms_k = dag_kernel_ms(ace, torch, G, tc, A, timed, 20, 5)
    fl = dag_flops_per_env(G.stats())["total"]
    return {"workload": f"{w.name}: {E} environments, {len(pos)} neighbour vectors, O(3), nu<={w.nu_max}, "
                        f"total degree<={w.degree_max}, n<={w.n_max}, l<={w.l_max}",
            "value": E / (ms * 1e-3), "ms_per_step": ms, "schedule_kind": G.schedule_kind(),
            "kernel_ms": ms_k, "frac": fl * E / (ms_k * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=5,
                    help="workload id (default 5: 8192 environments, nu<=6, D<=16, the largest basis)")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="environments of the oracle's CPU baseline and parity sample "
                         "(default: the whole batch up to 4096 environments, else 512)")
    ap.add_argument("--naive-steps", type=int, default=3,
                    help="timed steps of the naive baseline when one of its steps takes over 50 ms")
    ap.add_argument("--no-naive", action="store_true",
                    help="skip the naive baseline (for profiling runs)")
    ap.add_argument("--record-schedule", metavar="PATH",
                    help="write the schedule options the run applied to PATH (for the counter summaries)")
    ap.add_argument("--pmc-counters", nargs="+", metavar="DB",
                    help="reduce rocprofv3 counter databases of runs that wrote --record-schedule to "
                         "profiles/dag_kernel_counters_w<workload>.json and exit (needs --schedule-file)")
    ap.add_argument("--schedule-file", metavar="PATH", help="schedule options written by --record-schedule")
    ap.add_argument("--pmc-table", nargs="+", metavar="DB",
                    help="print the mean per dispatch of every counter in these rocprofv3 databases, "
                         "per kernel, as JSON, and exit")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 4096-environment phi+forces figures reported beside a larger workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--algorithm", type=int, default=1, choices=[1, 2],
                    help="insertion heuristic of the DAG (Algorithm 1 or 2)")
    ap.add_argument("--alg-n", type=int, default=2, help="Algorithm 2's parameter n")
    ap.add_argument("--degree-p", default="1", choices=["1", "2", "inf"],
                    help="degree notion of the basis: p-norm of the element degrees")
    ap.add_argument("--schedule", default="auto", choices=["auto", "forest", "remat", "layered"],
                    help="DAG kernel to use (auto: what the library picks, then autotuned)")
    ap.add_argument("--no-tune", action="store_true", help="skip the schedule autotuner")
    ap.add_argument("--retune", action="store_true", help="ignore cached and shipped tuned schedules")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of hipGraph replays")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, copy a buffer of this many MiB once (scale for HBM counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="reduce two rocprofv3 counter databases (FETCH_SIZE, WRITE_SIZE runs made with "
                         "--calibrate-copy) to profiles/dag_kernel_traffic_w<workload>.json and exit")
    args = ap.parse_args()
    if args.pmc_table:
        print(json.dumps(pmc_table(args.pmc_table), indent=1))
        return
    if args.pmc_summary or args.pmc_counters:
        with open(args.schedule_file) as f:
            rec = json.load(f)
        if rec["workload"] != args.workload or rec["source_hash"] != source_hash():
            raise SystemExit("the schedule file belongs to another workload or other sources")
        if args.pmc_counters:
            out = summarize_counters(args.pmc_counters, args.workload, rec["schedule"], counters_path(args.workload))
        else:
            out = summarize_pmc(args.pmc_summary[0], args.pmc_summary[1], args.calibrate_copy or 512, args.workload,
                                rec["schedule"], traffic_path(args.workload))
        print(json.dumps(out))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); environments are "
              "independent, so several GPUs would each run this same single-GPU pass on their own "
              "shard of the batch.", file=sys.stderr)
        sys.exit(2)

    w = wl.WORKLOADS[args.workload]
    off, pos = wl.batch(w)
    E, N = len(off) - 1, len(pos)

    cpu = None
    if args.degree_p != "1":
        args.no_cpu_baseline = True   # the oracle baseline lists the total-degree set
    if args.cpu_sample is None:
        args.cpu_sample = default_cpu_sample(args.workload)
    if not args.no_cpu_baseline:
        print(f"[bench] oracle CPU baseline on a {args.cpu_sample}-environment sample ...", file=sys.stderr,
              flush=True)
        s_envs, s_phi, s_grad, cpu = cpu_baseline(args.workload, off, pos, args.cpu_sample)
        print(f"[bench] oracle: {cpu['value']:.1f} env/s on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import torch
    import paper_2202_04140_amd as ace

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    degree_p = {"1": 1, "2": 2, "inf": math.inf}[args.degree_p]
    G = ace.Graph(w.nu_max, w.degree_max, w.n_max, w.l_max, r_cut=w.r_cut, algorithm=args.algorithm,
                  alg_n=args.alg_n if args.algorithm == 2 else 1, degree_p=degree_p, group=w.group,
                  k_max=w.k_max)
    t_build = time.perf_counter() - t0
    if args.schedule != "auto":
        G.set_schedule(schedule=args.schedule)
    stats = G.stats()
    c = wl.coefficients(w, G.k_degrees())
    tc = torch.from_numpy(c).to(dev)
    toff = torch.from_numpy(off).to(dev)
    tpos = torch.from_numpy(pos).to(dev)
    phi = torch.empty((E, 2), dtype=torch.float64, device=dev)
    grad = torch.empty((N, 3), dtype=torch.float64, device=dev)
    G.workspace(E, dev)
    print(f"[bench] graph built in {t_build:.2f} s: V={stats['n_nodes']} |K|={stats['n_k']}", file=sys.stderr,
          flush=True)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        return a.elapsed_time(b) / steps, wall

    def distribution(fn, reps, warmup):
        """Per-replay times (ms) from an event pair around each call: median, p10, p90."""
        for _ in range(warmup):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        t = np.array([a.elapsed_time(b) for a, b in ev])
        return dict(median=float(np.median(t)), p10=float(np.percentile(t, 10)), p90=float(np.percentile(t, 90)),
                    replays=reps)

    # schedule autotuning on this batch (setup, outside the timed region)
    A = ace.basis(G, toff, tpos)
    tuned = None
    if not args.no_tune:
        from paper_2202_04140_amd import autotune
        tuned = autotune.tune(G, tc, A, use_cache=not args.retune, verbose=args.retune,
                              kinds=None if args.schedule == "auto" else (args.schedule,))
        print(f"[bench] schedule {tuned['opts']} ({'cached' if tuned['cached'] else 'tuned'})",
              file=sys.stderr, flush=True)

    if args.record_schedule:
        with open(args.record_schedule, "w") as f:
            json.dump(dict(workload=args.workload, source_hash=source_hash(), schedule=G.get_schedule()), f)

    def step_dag():
        ace.eval_grad(G, tc, toff, tpos, out=(phi, grad))

    def step_naive():
        ace.eval_grad(G, tc, toff, tpos, naive=True, out=(phi, grad))

    def graphed(fn):
        """Capture one step in a hipGraph (after eager warm-up) and return its replay."""
        fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        torch.cuda.synchronize()
        return g.replay

    # whole path, DAG and naive: hipGraph replays of one step (eager beside)
    ms_dag_eager, _ = timed(step_dag, args.steps, args.warmup)
    ms_dag, wall = (ms_dag_eager, None) if args.eager else timed(graphed(step_dag), args.steps, args.warmup)
    print(f"[bench] DAG phi+forces: {ms_dag:.3f} ms/step (eager {ms_dag_eager:.3f})", file=sys.stderr, flush=True)
    dist = None
    if not args.eager:
        dist = distribution(graphed(step_dag), max(args.steps, 10) if ms_dag < 20 else args.steps, 2)
    phi_dag, grad_dag = phi.clone(), grad.clone()
    # the naive baseline: fewer steps where one takes long (the same hipGraph timing)
    ms_naive = None
    if not args.no_naive:
        t = time.perf_counter()
        step_naive()
        torch.cuda.synchronize()
        slow = time.perf_counter() - t > 0.05
        n_steps, n_warm = (args.naive_steps, 1) if slow else (args.steps, args.warmup)
        ms_naive_eager, _ = timed(step_naive, n_steps, 0 if slow else n_warm)
        ms_naive = ms_naive_eager if args.eager else timed(graphed(step_naive), n_steps, n_warm)[0]
        print(f"[bench] naive phi+forces: {ms_naive:.3f} ms/step ({n_steps} steps)", file=sys.stderr, flush=True)
        phi_naive, grad_naive = phi.clone(), grad.clone()
        ms_naive_kernel = naive_kernel_ms(ace, torch, G, tc, A, timed, n_steps, 1)
    ms_fwd, _ = timed(lambda: ace.eval(G, tc, toff, tpos, out=phi), args.steps, args.warmup)

    ms_kernel = dag_kernel_ms(ace, torch, G, tc, A, timed, args.steps, args.warmup)
    fl = dag_flops_per_env(stats)
    kind = G.schedule_kind()
    kernel_name = {"forest": "forest_kernel", "remat": "remat_kernel", "layered": "dag_kernel"}[kind] + \
        " (forward + reverse)"
    achieved = fl["total"] * E / (ms_kernel * 1e-3) / 1e12
    sched = G.get_schedule()
    prof = _profile(counters_path(args.workload), args.workload, sched)

    # parity of the timed results
    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    pd, gd = phi_dag.cpu().numpy(), grad_dag.cpu().numpy()
    parity = {}
    if ms_naive is not None:
        pn, gn = phi_naive.cpu().numpy(), grad_naive.cpu().numpy()
        parity = dict(dag_vs_naive_phi=rel(pd, pn), dag_vs_naive_grad=rel(gd, gn),
                      dag_vs_naive_per_env=per_env_errors(pd[:, 0] + 1j * pd[:, 1], pn[:, 0] + 1j * pn[:, 1],
                                                          gd, gn, off))
    if cpu is not None:
        rows = np.concatenate([np.arange(off[e], off[e + 1]) for e in s_envs])
        pc = pd[s_envs, 0] + 1j * pd[s_envs, 1]
        sub_off = np.zeros(len(s_envs) + 1, dtype=np.int64)
        np.cumsum(np.diff(off.astype(np.int64))[s_envs], out=sub_off[1:])
        parity.update(oracle_phi=rel(pc, s_phi), oracle_grad=rel(gd[rows], s_grad),
                      oracle_sample=int(len(s_envs)),
                      oracle_per_env=per_env_errors(pc, s_phi, gd[rows], s_grad, sub_off))
    extra = None
    if not args.no_extra and args.workload != 3:
        extra = small_workload_figures(ace, torch, dev, timed, graphed, args)

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    out = {
        "metric": METRIC,
        "value": E / (ms_dag * 1e-3),
        "unit": "environments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_dag,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {E} environments, {N} neighbour vectors, "
                               f"{['O(3)', 'torus', 'SO(2)'][w.group]}, nu<={w.nu_max}, "
                               f"{'total degree' if degree_p == 1 else f'degree p={args.degree_p}'}<={w.degree_max}, "
                               + ("" if w.group == 1 else f"n<={w.n_max}, {'l' if w.group == 0 else '|m|'}<={w.l_max}, ")
                               + (f"feature k<={w.k_max} (4 species), " if w.k_max else "")
                               + f"Algorithm {args.algorithm}"
                               + (f" (n={args.alg_n})" if args.algorithm == 2 else ""),
                   "n_env": E, "n_nbr": N, "nu_max": w.nu_max, "degree_max": w.degree_max,
                   "n_max": w.n_max, "l_max": w.l_max},
        "naive": None if ms_naive is None else {
            "value": E / (ms_naive * 1e-3), "ms_per_step": ms_naive, "kernel_ms": ms_naive_kernel,
            "frac": naive_flops_per_env(stats)["total"] * E / (ms_naive_kernel * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "flops_per_env": naive_flops_per_env(stats)},
        "dag_vs_naive": None if ms_naive is None else ms_naive / ms_dag,
        "forces_per_s": N / (ms_dag * 1e-3),
        "phi_only_env_per_s": E / (ms_fwd * 1e-3),
        "roofline": {"bound": "alu", "kernel": kernel_name, "achieved": achieved,
                     "flops": "DAG count per environment (forward 6S+3T+2|K|, reverse 16S+8T), "
                              "a DAG-equivalent rate: the remat kernel recomputes parents and "
                              "evaluates one tuple per conjugate pair",
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": profiled_traffic(args.workload, sched), "kernel_ms": ms_kernel,
                     "flops_per_env": fl,
                     "executed": None if prof is None or "fp64_flops_per_launch" not in prof else {
                         "fp64_flops_per_launch": prof["fp64_flops_per_launch"],
                         "achieved": prof["fp64_flops_per_launch"] / (ms_kernel * 1e-3) / 1e12,
                         "frac": prof["fp64_flops_per_launch"] / (ms_kernel * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                         "valu_busy": prof.get("valu_busy"), "lds_active": prof.get("lds_active"),
                         "lds_bank_conflict_share": prof.get("lds_bank_conflict_share"),
                         "note": "FP64 VALU operations the kernel executes (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes, "
                                 "committed counter profile of this schedule) over the launch time"}},
        "eager_ms_per_step": ms_dag_eager,
        "step_ms_distribution": dist,
        "timing": "eager launches" if args.eager else "hipGraph replays of one captured step",
        "schedule": G.get_schedule(),
        "schedule_kind": kind,
        "cpu_baseline": cpu,
        "parity": parity,
        "graph_build_s": t_build,
        "w3": extra,
        "dag": {"V": stats["n_nodes"], "K": stats["n_k"], "aux": stats["n_aux"], "stored": stats["n_stored"],
                "childless": stats["n_childless"]},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
