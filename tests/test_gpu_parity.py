"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (norm-wise over the batch, complex values for phi and A):
  A    <= 1e-13      (one-particle basis; ~P1 * J roundings of O(1) terms)
  phi  <= 1e-11      (stated target)
  Abar <= 1e-11      (same arithmetic depth as phi)
  grad <= 1e-9       (stated target for forces)
The same seeded inputs go to both sides; the oracle computes its own K,
one-particle list and coefficients' degrees.
"""

import math

import numpy as np
import pytest

import workloads as wl
from oracle import contraction as oc
from oracle import onebody as ob
from oracle.indexsets import all_invariant_tuples, group_o3

pytestmark = pytest.mark.gpu

TOL_A, TOL_PHI, TOL_ABAR, TOL_GRAD = 1e-13, 1e-11, 1e-11, 1e-9


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def per_env_max(phi, phi_ref, grad, grad_ref, offsets):
    """Largest per-environment relative errors: |phi_e - ref_e| / |ref_e| over the
    environments with |ref_e| >= 1e-6 RMS(ref) (the others are only counted), and
    ||g_e - ref_e|| / ||ref_e|| over each environment's gradient rows."""
    phi, phi_ref = np.asarray(phi), np.asarray(phi_ref)
    mag = np.abs(phi_ref)
    ok = mag >= 1e-6 * np.sqrt(np.mean(mag ** 2))
    e_phi = float(np.max(np.abs(phi - phi_ref)[ok] / mag[ok])) if ok.any() else 0.0
    e_g = 0.0
    off = np.asarray(offsets, dtype=np.int64)
    for e in range(len(off) - 1):
        a, b = off[e], off[e + 1]
        nr = np.linalg.norm(grad_ref[a:b])
        if b > a and nr > 0:
            e_g = max(e_g, float(np.linalg.norm(grad[a:b] - grad_ref[a:b]) / nr))
    return e_phi, e_g, int((~ok).sum())


_ORACLE = {}
_GRAPH = {}


def oracle_basis(wid):
    """(group, K, c) from the oracle's own enumeration (cached)."""
    if wid not in _ORACLE:
        w = wl.WORKLOADS[wid]
        g = group_o3(w.n_max, w.l_max, w.degree_max)
        K = all_invariant_tuples(g, w.nu_max, w.degree_max)
        c = wl.coefficients(w, np.array([g.degree(k) for k in K]))
        _ORACLE[wid] = (g, K, c)
    return _ORACLE[wid]


def graph(wid, device, schedule=None):
    """The library graph of a workload (cached), optionally with a forced schedule."""
    import paper_2202_04140_amd as ace
    if (wid, schedule) not in _GRAPH:
        w = wl.WORKLOADS[wid]
        G = ace.Graph(w.nu_max, w.degree_max, w.n_max, w.l_max, r_cut=w.r_cut)
        if schedule is not None:
            G.set_schedule(schedule=schedule)
        g, K, _ = oracle_basis(wid)
        kt = G.k_tuples()
        assert kt.shape[0] == len(K)
        for q in (0, len(K) // 3, len(K) - 1):
            assert tuple(x for x in kt[q] if x >= 0) == K[q]
        _GRAPH[(wid, schedule)] = G
    return _GRAPH[(wid, schedule)]


def to_dev(device, *arrs):
    import torch
    out = []
    for a in arrs:
        if a.dtype == np.int32:
            out.append(torch.from_numpy(np.ascontiguousarray(a)).to(device))
        else:
            out.append(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device))
    return out


def cplx(t):
    a = t.detach().cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def problem(wid, n_env=None, envs=None):
    w = wl.WORKLOADS[wid]
    off, pos = wl.batch(w)
    if envs is None and n_env is not None:
        envs = wl.subset(off, n_env)
    if envs is not None:
        off, pos = wl.gather(off, pos, envs)
    return off, pos


# ---- one-particle basis ------------------------------------------------------------
@pytest.mark.parametrize("wid,n_env", [(1, None), (2, 64), (4, 32), (5, 8)])
def test_basis_parity(device, wid, n_env):
    import paper_2202_04140_amd as ace
    print(f"basis wid={wid} n_env={n_env}", flush=True)
    G = graph(wid, device)
    g, _, _ = oracle_basis(wid)
    off, pos = problem(wid, n_env)
    toff, tpos = to_dev(device, off, pos)
    A = cplx(ace.basis(G, toff, tpos))
    ref = ob.pooled_A(g.labels, off, pos, wl.WORKLOADS[wid].r_cut)
    assert rel(A, ref) <= TOL_A


# ---- contraction alone, from random one-particle values ----------------------------
# call flags and forced schedule of each evaluation mode
MODES = {"dag": ({}, None), "remat": ({}, "remat"), "layered": ({"layered": True}, None),
         "naive": ({"naive": True}, None)}


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("wid,n_env", [(1, 16), (2, 48), (4, 6)])
def test_contract_random_A(device, wid, n_env, mode):
    import paper_2202_04140_amd as ace
    print(f"contract wid={wid} n_env={n_env} mode={mode}", flush=True)
    kw, sched = MODES[mode]
    G = graph(wid, device, sched)
    g, K, c = oracle_basis(wid)
    A = wl.random_A(n_env, len(g), seed=100 + wid) * 0.5
    At = np.stack([A.real, A.imag], -1)
    tc, tA = to_dev(device, c, At)
    phi, Ab = ace.contract(G, tc, tA, with_grad=True, **kw)
    phi_ref = oc.phi_naive(K, c, A)
    ab_ref = oc.abar_naive(K, c, A)
    assert rel(cplx(phi), phi_ref) <= TOL_PHI
    assert rel(cplx(Ab), ab_ref) <= TOL_ABAR
    # forward-only launch gives the same phi
    phi2 = ace.contract(G, tc, tA, with_grad=False, **kw)
    assert rel(cplx(phi2), phi_ref) <= TOL_PHI


def test_schedule_in_use(device):
    assert graph(1, device).schedule_kind() == "forest"
    assert graph(3, device).schedule_kind() == "forest"
    assert graph(4, device).schedule_kind() == "forest"
    assert graph(5, device).schedule_kind() == "remat"
    assert graph(2, device, "remat").schedule_kind() == "remat"


# ---- two environments per forest block ----------------------------------------------
@pytest.mark.parametrize("wid,n_env", [(1, 15), (2, 33), (3, 17), (4, 5)])
def test_forest_two_envs_per_block(device, wid, n_env):
    """env_per_block = 2 (two environments share every schedule and coefficient
    load; an odd count leaves the last block half empty; a basis whose two
    environments do not fit in LDS falls back to one): contract with and without
    folding, forward only, and the full path, against the oracle."""
    import paper_2202_04140_amd as ace
    print(f"forest two envs wid={wid} n_env={n_env}", flush=True)
    w = wl.WORKLOADS[wid]
    G = ace.Graph(w.nu_max, w.degree_max, w.n_max, w.l_max, r_cut=w.r_cut)
    G.set_schedule(schedule="forest", env_per_block=2)
    assert G.schedule_kind() == "forest" and G.get_schedule()["env_per_block"] == 2
    g, K, c = oracle_basis(wid)
    A = wl.random_A(n_env, len(g), seed=400 + wid) * 0.5
    tc, tA = to_dev(device, c, np.stack([A.real, A.imag], -1))
    phi_ref, ab_ref = oc.phi_naive(K, c, A), oc.abar_naive(K, c, A)
    phi, Ab = ace.contract(G, tc, tA, with_grad=True)
    assert rel(cplx(phi), phi_ref) <= TOL_PHI
    assert rel(cplx(Ab), ab_ref) <= TOL_ABAR
    assert rel(cplx(ace.contract(G, tc, tA, with_grad=False)), phi_ref) <= TOL_PHI
    As = wl.random_A_conj(n_env, g.labels, 500 + wid) * 0.5
    dA = wl.random_A_conj(n_env, g.labels, 600 + wid)
    (tAs,) = to_dev(device, np.stack([As.real, As.imag], -1))
    phis_ref, abs_ref = oc.phi_naive(K, c, As), oc.abar_naive(K, c, As)
    phi, Ab = ace.contract(G, tc, tAs, with_grad=True, conj_symmetric=True)
    assert rel(cplx(phi), phis_ref) <= TOL_PHI
    lhs = np.real(np.sum(cplx(Ab) * dA, axis=1))
    rhs = np.real(np.sum(abs_ref * dA, axis=1))
    assert rel(lhs, rhs) <= TOL_ABAR
    assert rel(cplx(ace.contract(G, tc, tAs, with_grad=False, conj_symmetric=True)), phis_ref) <= TOL_PHI
    if wid in (1, 3):
        off, pos = problem(wid, n_env)
        tc, toff, tpos = to_dev(device, c, off, pos)
        phi, grad = ace.eval_grad(G, tc, toff, tpos)
        phi_ref, g_ref = oc.grad_naive(g.labels, K, c, off, pos, w.r_cut)
        assert rel(cplx(phi), phi_ref) <= TOL_PHI
        assert rel(grad.cpu().numpy(), g_ref) <= TOL_GRAD


# ---- remat schedule: two environments per block, 1024-thread blocks -----------------
@pytest.mark.parametrize("spec,n_env,bt,ne", [((1,), 15, 1024, 2), ((3,), 17, 512, 2), ((2,), 33, 1024, 1),
                                              ((6, 10, 3, 3), 9, 1024, 2), ((6, 10, 3, 3), 8, 256, 2)])
def test_remat_envs_per_block(device, spec, n_env, bt, ne):
    """The remat kernel with env_per_block = 2 (two environments share every
    metadata and coefficient load; an odd count leaves the last block half
    empty) and block sizes up to 1024: contract with and without folding,
    forward only, and the full path, against the oracle."""
    import paper_2202_04140_amd as ace
    print(f"remat envs per block spec={spec} n_env={n_env} block={bt} ne={ne}", flush=True)
    if len(spec) == 1:
        w = wl.WORKLOADS[spec[0]]
        nu, D, nmax, lmax, seed = w.nu_max, w.degree_max, w.n_max, w.l_max, spec[0]
        g, K, c = oracle_basis(spec[0])
    else:
        nu, D, nmax, lmax = spec
        seed = 77
        g = group_o3(nmax, lmax, D)
        K = all_invariant_tuples(g, nu, D)
        c = np.random.default_rng(seed).standard_normal(len(K)) / (1.0 + np.array([g.degree(k) for k in K])) ** 2
    G = ace.Graph(nu, D, nmax, lmax)
    G.set_schedule(schedule="remat", env_per_block=ne, block_threads=bt)
    assert G.schedule_kind() == "remat" and G.get_schedule()["env_per_block"] == ne
    A = wl.random_A(n_env, len(g), seed=700 + seed) * 0.5
    tc, tA = to_dev(device, c, np.stack([A.real, A.imag], -1))
    phi_ref, ab_ref = oc.phi_naive(K, c, A), oc.abar_naive(K, c, A)
    phi, Ab = ace.contract(G, tc, tA, with_grad=True)
    assert rel(cplx(phi), phi_ref) <= TOL_PHI
    assert rel(cplx(Ab), ab_ref) <= TOL_ABAR
    assert rel(cplx(ace.contract(G, tc, tA, with_grad=False)), phi_ref) <= TOL_PHI
    As = wl.random_A_conj(n_env, g.labels, 800 + seed) * 0.5
    dA = wl.random_A_conj(n_env, g.labels, 900 + seed)
    (tAs,) = to_dev(device, np.stack([As.real, As.imag], -1))
    phis_ref, abs_ref = oc.phi_naive(K, c, As), oc.abar_naive(K, c, As)
    phi, Ab = ace.contract(G, tc, tAs, with_grad=True, conj_symmetric=True)
    assert rel(cplx(phi), phis_ref) <= TOL_PHI
    lhs = np.real(np.sum(cplx(Ab) * dA, axis=1))
    rhs = np.real(np.sum(abs_ref * dA, axis=1))
    assert rel(lhs, rhs) <= TOL_ABAR
    assert rel(cplx(ace.contract(G, tc, tAs, with_grad=False, conj_symmetric=True)), phis_ref) <= TOL_PHI
    off, pos = problem(3, n_env)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi, grad = ace.eval_grad(G, tc, toff, tpos)
    phi_ref, g_ref = oc.grad_naive(g.labels, K, c, off, pos, 5.0)
    assert rel(cplx(phi), phi_ref) <= TOL_PHI
    assert rel(grad.cpu().numpy(), g_ref) <= TOL_GRAD


# ---- full path ---------------------------------------------------------------------
@pytest.mark.parametrize("naive", [False, True])
@pytest.mark.parametrize("wid,n_env", [(1, None), (2, 96)])
def test_eval_parity(device, wid, n_env, naive):
    import paper_2202_04140_amd as ace
    print(f"eval wid={wid} n_env={n_env} naive={naive}", flush=True)
    G = graph(wid, device)
    g, K, c = oracle_basis(wid)
    off, pos = problem(wid, n_env)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi = cplx(ace.eval(G, tc, toff, tpos, naive=naive, check=True))
    ref = oc.eval_naive(g.labels, K, c, off, pos, wl.WORKLOADS[wid].r_cut)
    assert rel(phi, ref) <= TOL_PHI


@pytest.mark.parametrize("unfolded", [False, True])
@pytest.mark.parametrize("mode", ["dag", "remat", "layered"])
@pytest.mark.parametrize("wid,n_env", [(3, 40), (4, 10)])
def test_forward_only_every_schedule(device, wid, n_env, mode, unfolded):
    """ace_eval (no reverse pass) in each schedule, conjugate pairs folded or not.
    Its coefficients are gathered on the basis kernel's grid for the forward-only
    schedule (another gather map than the one with the reverse pass); phi matches
    the oracle and the phi of ace_eval_grad."""
    import paper_2202_04140_amd as ace
    print(f"forward only wid={wid} n_env={n_env} mode={mode} unfolded={unfolded}", flush=True)
    kw, sched = MODES[mode]
    G = graph(wid, device, sched)
    g, K, c = oracle_basis(wid)
    off, pos = problem(wid, n_env)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi = cplx(ace.eval(G, tc, toff, tpos, unfolded=unfolded, **kw))
    phi_g, _ = ace.eval_grad(G, tc, toff, tpos, unfolded=unfolded, **kw)
    ref = oc.eval_naive(g.labels, K, c, off, pos, wl.WORKLOADS[wid].r_cut)
    assert rel(phi, ref) <= TOL_PHI
    assert rel(phi, cplx(phi_g)) <= TOL_PHI


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("wid,n_env", [(1, None), (3, 64), (4, 12)])
def test_eval_grad_parity(device, wid, n_env, mode):
    import paper_2202_04140_amd as ace
    print(f"eval_grad wid={wid} n_env={n_env} mode={mode}", flush=True)
    kw, sched = MODES[mode]
    G = graph(wid, device, sched)
    g, K, c = oracle_basis(wid)
    off, pos = problem(wid, n_env)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi, grad = ace.eval_grad(G, tc, toff, tpos, **kw)
    phi_ref, g_ref = oc.grad_naive(g.labels, K, c, off, pos, wl.WORKLOADS[wid].r_cut)
    assert rel(cplx(phi), phi_ref) <= TOL_PHI
    assert rel(grad.cpu().numpy(), g_ref) <= TOL_GRAD


def test_full_size_sampled_and_dag_vs_naive(device):
    """Workload 3 at full size, in the launch configuration the benchmark times;
    24 sampled environments (incl. the smallest and largest) against the oracle,
    and every environment DAG against naive."""
    import paper_2202_04140_amd as ace
    wid = 3
    G = graph(wid, device)
    g, K, c = oracle_basis(wid)
    off, pos = problem(wid)
    print(f"full size wid=3 n_env={len(off) - 1}", flush=True)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi, grad = ace.eval_grad(G, tc, toff, tpos)
    phi_n, grad_n = ace.eval_grad(G, tc, toff, tpos, naive=True)
    phi, grad, phi_n, grad_n = cplx(phi), grad.cpu().numpy(), cplx(phi_n), grad_n.cpu().numpy()
    assert rel(phi, phi_n) <= TOL_PHI
    assert rel(grad, grad_n) <= TOL_GRAD
    envs = wl.subset(off, 24)
    so, sp_ = wl.gather(off, pos, envs)
    phi_ref, g_ref = oc.grad_naive(g.labels, K, c, so, sp_, wl.WORKLOADS[wid].r_cut)
    rows = np.concatenate([np.arange(off[e], off[e + 1]) for e in envs])
    assert rel(phi[envs], phi_ref) <= TOL_PHI
    assert rel(grad[rows], g_ref) <= TOL_GRAD


def stored_oracle_sample(wid, off, pos, c):
    """The oracle's phi and gradients on a seeded subset of a workload, written by
    tests/golden/make_oracle_samples.py (oracle only); the inputs are checked
    against the fingerprint stored with them."""
    import os
    import sys
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    from make_oracle_samples import fingerprint, path_for
    d = np.load(path_for(wid))
    envs = d["envs"]
    so, sp_ = wl.gather(off, pos, envs)
    assert np.array_equal(so, d["offsets"])
    assert str(d["fingerprint"]) == fingerprint(sp_, c), "inputs differ from those of the stored oracle values"
    return envs, so, d["phi"], d["grad"]


@pytest.mark.parametrize("wid,n_sample", [(3, 24), (4, 64), (5, 64)])
def test_full_size_in_benchmark_schedule(device, wid, n_sample, tmp_path, monkeypatch):
    """Every environment of the 4096-, 32768- and 8192-environment workloads in one
    ace_eval_grad call, in the schedule the benchmark applies to that batch (the
    shipped autotuned choice: an empty user cache, as on a fresh machine); sampled
    environments (the smallest and largest neighbour counts among them) against the
    oracle (live for the 4096-environment basis, stored oracle values for the two
    larger ones), all of them against the naive kernel; norm-wise over the batch
    and per environment."""
    import paper_2202_04140_amd as ace
    from paper_2202_04140_amd import autotune
    monkeypatch.setenv("ACE_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    w = wl.WORKLOADS[wid]
    G = ace.Graph(w.nu_max, w.degree_max, w.n_max, w.l_max, r_cut=w.r_cut)
    off, pos = problem(wid)
    c = wl.coefficients(w, G.k_degrees())
    print(f"full size wid={wid} n_env={len(off) - 1} n_nbr={len(pos)}", flush=True)
    tc, toff, tpos = to_dev(device, c, off, pos)
    tuned = autotune.tune(G, tc, ace.basis(G, toff, tpos))
    assert tuned["cached"], "no shipped schedule for this workload"
    assert G.schedule_kind() == tuned["opts"]["schedule"]
    phi, grad = ace.eval_grad(G, tc, toff, tpos)
    phi_n, grad_n = ace.eval_grad(G, tc, toff, tpos, naive=True)
    phi, grad, phi_n, grad_n = cplx(phi), grad.cpu().numpy(), cplx(phi_n), grad_n.cpu().numpy()
    assert np.isfinite(phi).all() and np.isfinite(grad).all()
    assert rel(phi, phi_n) <= TOL_PHI
    assert rel(grad, grad_n) <= TOL_GRAD
    e_phi, e_g, _ = per_env_max(phi, phi_n, grad, grad_n, off)
    assert e_phi <= TOL_PHI and e_g <= TOL_GRAD
    J = np.diff(off)
    if wid == 3:
        g, K, c_or = oracle_basis(wid)
        assert np.array_equal(c_or, c)
        envs = wl.subset(off, n_sample)
        so, sp_ = wl.gather(off, pos, envs)
        phi_ref, g_ref = oc.grad_naive(g.labels, K, c, so, sp_, w.r_cut)
    else:
        envs, so, phi_ref, g_ref = stored_oracle_sample(wid, off, pos, c)
    assert len(envs) == n_sample
    assert J[envs].min() == J.min() and J[envs].max() == J.max()
    rows = np.concatenate([np.arange(off[e], off[e + 1]) for e in envs])
    assert rel(phi[envs], phi_ref) <= TOL_PHI
    assert rel(grad[rows], g_ref) <= TOL_GRAD
    e_phi, e_g, _ = per_env_max(phi[envs], phi_ref, grad[rows], g_ref, so)
    assert e_phi <= TOL_PHI and e_g <= TOL_GRAD


# ---- edge cases ----------------------------------------------------------------------
def test_edge_cases_empty_ragged(device):
    import paper_2202_04140_amd as ace
    import torch
    wid = 1
    G = graph(wid, device)
    g, K, c = oracle_basis(wid)
    # empty batch: no-op
    tc, = to_dev(device, c)
    z = torch.zeros(1, dtype=torch.int32, device=device)
    p0 = torch.zeros((0, 3), dtype=torch.float64, device=device)
    assert ace.eval(G, tc, z, p0).shape == (0, 2)
    # environments with 0, 1, 2 and many neighbours
    counts = [0, 1, 2, 0, 37, 1, 64]
    off = np.zeros(len(counts) + 1, np.int32)
    off[1:] = np.cumsum(counts)
    pos = wl.positions(int(off[-1]), 77)
    toff, tpos = to_dev(device, off, pos)
    for naive in (False, True):
        phi, grad = ace.eval_grad(G, tc, toff, tpos, naive=naive)
        phi_ref, g_ref = oc.grad_naive(g.labels, K, c, off, pos, 5.0)
        phi = cplx(phi)
        assert phi[0] == 0 and phi[3] == 0
        assert rel(phi, phi_ref) <= TOL_PHI
        assert rel(grad.cpu().numpy(), g_ref) <= TOL_GRAD


def test_invalid_offsets_rejected_with_check(device):
    """ACE_FLAG_CHECK validates the offsets on the device (no synchronisation in
    the call, so it can be captured); the result is read from the workspace
    afterwards.  Invalid offsets make the launches that read them do nothing."""
    import paper_2202_04140_amd as ace
    import torch
    G = graph(1, device)
    _, _, c = oracle_basis(1)
    off = np.array([0, 5, 3], np.int32)   # decreasing
    pos = wl.positions(5, 78)
    tc, toff, tpos = to_dev(device, c, off, pos)
    with pytest.raises((ace.AceError, ValueError)):   # binding check
        ace.eval(G, tc, toff, tpos, check=True)
    lib = ace.lib()
    phi = torch.empty((2, 2), dtype=torch.float64, device=device)
    grad = torch.full((5, 3), 7.0, dtype=torch.float64, device=device)
    ws = G.workspace(2, device, ace.FLAG_CHECK)
    # the library's own check without the binding in front
    for bad, msg in (([0, 5, 3], b"non-decreasing"), ([1, 3, 5], b"offsets[0]")):
        toff.copy_(torch.tensor(bad, dtype=torch.int32))
        st = lib.ace_eval(G.handle, tc.data_ptr(), 2, toff.data_ptr(), tpos.data_ptr(), phi.data_ptr(),
                          ws.data_ptr(), ws.numel(), ace.FLAG_CHECK, ace._stream(device))
        assert st == 0
        torch.cuda.synchronize()
        assert lib.ace_check_offsets_result(ws.data_ptr()) == 1 and msg in lib.ace_last_error()
    # inside a captured graph: the same launch sequence, replayed with valid
    # and with invalid offsets (written between replays)
    toff.copy_(torch.tensor([0, 2, 5], dtype=torch.int32))
    def call():
        st = lib.ace_eval_grad(G.handle, tc.data_ptr(), 2, toff.data_ptr(), tpos.data_ptr(), phi.data_ptr(),
                               grad.data_ptr(), ws.data_ptr(), ws.numel(), ace.FLAG_CHECK, ace._stream(device))
        assert st == 0
    call()
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        call()
    torch.cuda.synchronize()
    g, K, _ = oracle_basis(1)
    for valid in (True, False, True):
        toff.copy_(torch.tensor([0, 2, 5] if valid else [0, 5, 3], dtype=torch.int32))
        grad.fill_(7.0)
        gr.replay()
        torch.cuda.synchronize()
        st = lib.ace_check_offsets_result(ws.data_ptr())
        if valid:
            assert st == 0
            _, g_ref = oc.grad_naive(g.labels, K, c, np.array([0, 2, 5]), pos, 5.0)
            assert rel(grad.cpu().numpy(), g_ref) <= TOL_GRAD
        else:
            assert st == 1 and b"non-decreasing" in lib.ace_last_error()
            assert torch.all(grad == 7.0)   # the gradient launch read nothing


def test_workspace_too_small_is_an_error(device):
    import ctypes
    import paper_2202_04140_amd as ace
    import torch
    G = graph(1, device)
    _, _, c = oracle_basis(1)
    off, pos = problem(1)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi = torch.empty((16, 2), dtype=torch.float64, device=device)
    ws = torch.empty(64, dtype=torch.uint8, device=device)
    st = ace.lib().ace_eval(G.handle, tc.data_ptr(), 16, toff.data_ptr(), tpos.data_ptr(), phi.data_ptr(),
                            ws.data_ptr(), 64, 0, None)
    assert st == 1
    assert b"workspace too small" in ace.lib().ace_last_error()


# ---- gradient against central differences of the GPU path ---------------------------
def test_gradient_central_differences(device):
    import paper_2202_04140_amd as ace
    import torch
    wid = 3
    G = graph(wid, device)
    _, _, c = oracle_basis(wid)
    off, pos = problem(wid, 8)
    tc, toff = to_dev(device, c, off)
    tpos, = to_dev(device, pos)
    _, grad = ace.eval_grad(G, tc, toff, tpos)
    grad = grad.cpu().numpy()
    h = 1e-6
    J = np.diff(off)
    fd = np.zeros_like(pos)
    for jj in range(int(J.max())):
        envs = np.nonzero(J > jj)[0]
        rows = off[envs] + jj
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[rows, d] += h
            pm[rows, d] -= h
            fp = ace.eval(G, tc, toff, torch.from_numpy(pp).to(device))[:, 0].cpu().numpy()
            fm = ace.eval(G, tc, toff, torch.from_numpy(pm).to(device))[:, 0].cpu().numpy()
            fd[rows, d] = (fp[envs] - fm[envs]) / (2 * h)
    assert rel(grad, fd) <= 1e-6


# ---- symmetries and determinism on the device ----------------------------------------
def test_invariance_and_determinism(device):
    import paper_2202_04140_amd as ace
    import torch
    wid = 3
    G = graph(wid, device)
    _, _, c = oracle_basis(wid)
    off, pos = problem(wid, 32)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi0 = cplx(ace.eval(G, tc, toff, tpos))
    phi1 = cplx(ace.eval(G, tc, toff, tpos))
    assert np.array_equal(phi0, phi1)                 # forward pass has a fixed order
    a = 0.61
    Q = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    phiq = cplx(ace.eval(G, tc, toff, torch.from_numpy(pos @ Q.T).to(device)))
    assert rel(phiq, phi0) <= 1e-12
    phii = cplx(ace.eval(G, tc, toff, torch.from_numpy(-pos).to(device)))
    assert rel(phii, phi0) <= 1e-12
    rng = np.random.default_rng(0)
    perm = np.concatenate([off[e] + rng.permutation(off[e + 1] - off[e]) for e in range(len(off) - 1)])
    phip = cplx(ace.eval(G, tc, toff, torch.from_numpy(pos[perm]).to(device)))
    assert rel(phip, phi0) <= 1e-12


# ---- gradients on and near the z-axis (theta = 0, pi) --------------------------------
def test_gradient_at_and_near_the_poles(device):
    """Neighbours exactly on +-z and at angles 1e-12, 1e-8 and 1e-4 from it, beside
    random ones: the gradient (Cartesian recurrences, no division by sin(theta))
    against differences of the oracle's phi, which is smooth there: a central
    difference with h = 1e-6 within 1e-6 and a five-point stencil with h = 1e-3
    within 1e-8, and against the oracle's gradient within 1e-9 where
    sin(theta) >= 1e-4 (the oracle's gradient divides by sin(theta))."""
    import paper_2202_04140_amd as ace
    wid = 1
    w = wl.WORKLOADS[wid]
    G = graph(wid, device)
    g, K, c = oracle_basis(wid)
    rng = np.random.default_rng(11)
    special = []
    for sign in (1.0, -1.0):
        for delta in (0.0, 1e-12, 1e-8, 1e-4):
            r = rng.uniform(1.0, 4.5)
            beta = rng.uniform(-np.pi, np.pi)
            special.append(r * np.array([math.sin(delta) * math.cos(beta), math.sin(delta) * math.sin(beta),
                                         sign * math.cos(delta)]))
    # one environment per special neighbour, with three random neighbours beside it
    others = wl.positions(3 * len(special), 91)
    pos = np.concatenate([np.concatenate([sp[None, :], others[3 * i:3 * i + 3]]) for i, sp in enumerate(special)])
    off = np.arange(0, 4 * len(special) + 1, 4, dtype=np.int32)
    print(f"poles: {len(special)} environments", flush=True)
    tc, toff, tpos = to_dev(device, c, off, pos)
    _, grad = ace.eval_grad(G, tc, toff, tpos)
    grad = grad.cpu().numpy()
    assert np.isfinite(grad).all()
    rows = off[:-1]                                   # the special neighbour of each environment

    def phi_re(p):
        return oc.eval_naive(g.labels, K, c, off, p, w.r_cut).real

    def diff(h, stencil):
        out = np.zeros((len(rows), 3))
        for d in range(3):
            acc = np.zeros(len(rows))
            for wgt, step in stencil:
                p = pos.copy()
                p[rows, d] += step * h
                acc += wgt * phi_re(p)
            out[:, d] = acc / h
        return out

    g_cd = diff(1e-6, [(0.5, 1.0), (-0.5, -1.0)])
    g_5p = diff(1e-3, [(-1 / 12, 2.0), (2 / 3, 1.0), (-2 / 3, -1.0), (1 / 12, -2.0)])
    assert rel(grad[rows], g_cd) <= 1e-6
    assert rel(grad[rows], g_5p) <= 1e-8
    for i in range(len(rows)):
        assert np.linalg.norm(grad[rows[i]] - g_5p[i]) <= 1e-8 * np.linalg.norm(g_5p), i
    # oracle gradient where sin(theta) >= 1e-4 for every neighbour of the environment
    far = [i for i in range(len(special)) if np.hypot(*special[i][:2]) >= 0.99e-4 * np.linalg.norm(special[i])]
    assert len(far) == 2
    for i in far:
        so = np.array([0, 4], dtype=np.int32)
        _, g_ref = oc.grad_naive(g.labels, K, c, so, pos[4 * i:4 * i + 4], w.r_cut)
        assert rel(grad[4 * i:4 * i + 4], g_ref) <= TOL_GRAD


@pytest.mark.parametrize("wid,n_env", [(3, 256), (5, 16)])
def test_eval_grad_repeatable(device, wid, n_env):
    """The same ace_eval_grad call twice: phi is bitwise repeatable (fixed
    summation order); the reverse pass adds adjoints with LDS atomics in an
    order that may change from run to run, so the gradients are compared within
    1e-13 (norm-wise and per environment), far below the 1e-9 target."""
    import paper_2202_04140_amd as ace
    w = wl.WORKLOADS[wid]
    G = graph(wid, device)
    c = wl.coefficients(w, G.k_degrees())
    off, pos = problem(wid, n_env)
    print(f"repeat wid={wid} n_env={n_env}", flush=True)
    tc, toff, tpos = to_dev(device, c, off, pos)
    runs = [ace.eval_grad(G, tc, toff, tpos) for _ in range(3)]
    phis = [cplx(p) for p, _ in runs]
    grads = [gr.cpu().numpy() for _, gr in runs]
    for k in (1, 2):
        assert np.array_equal(phis[k], phis[0])
        assert rel(grads[k], grads[0]) <= 1e-13
        assert per_env_max(phis[k], phis[0], grads[k], grads[0], off)[1] <= 1e-13


def test_autograd_function(device):
    import paper_2202_04140_amd as ace
    import torch
    wid = 1
    G = graph(wid, device)
    _, _, c = oracle_basis(wid)
    off, pos = problem(wid)
    tc, toff, tpos = to_dev(device, c, off, pos)
    p = tpos.clone().requires_grad_(True)
    e = ace.AceEnergy.apply(p, toff, tc, G)
    w = torch.linspace(-1, 1, e.shape[0], dtype=torch.float64, device=device)
    (e * w).sum().backward()
    _, grad = ace.eval_grad(G, tc, toff, tpos)
    counts = (toff[1:] - toff[:-1]).long()
    ref = grad * torch.repeat_interleave(w, counts)[:, None]
    # separate launches: the reverse pass accumulates with atomics, so allow rounding
    assert torch.allclose(p.grad, ref, rtol=1e-12, atol=1e-14 * ref.abs().max().item())
    phi = ace.eval(G, tc, toff, tpos)
    assert torch.allclose(e.detach(), phi[:, 0], rtol=1e-14, atol=0)


# ---- large bases, sampled ----------------------------------------------------------------
@pytest.mark.parametrize("wid,n_env", [(4, 16), (5, 3)])
def test_large_basis_eval_grad(device, wid, n_env):
    import paper_2202_04140_amd as ace
    print(f"large wid={wid} n_env={n_env}", flush=True)
    G = graph(wid, device)
    g, K, c = oracle_basis(wid)
    off, pos = problem(wid, n_env)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi, grad = ace.eval_grad(G, tc, toff, tpos)
    phi_ref, g_ref = oc.grad_naive(g.labels, K, c, off, pos, wl.WORKLOADS[wid].r_cut)
    assert rel(cplx(phi), phi_ref) <= TOL_PHI
    assert rel(grad.cpu().numpy(), g_ref) <= TOL_GRAD


# ---- conjugate-pair folding (remat and forest schedules) -----------------------------
@pytest.mark.parametrize("sched", ["remat", None])
@pytest.mark.parametrize("wid,n_env", [(3, 40), (4, 24), (5, 4)])
def test_folded_and_unfolded_eval_grad_agree(device, wid, n_env, sched):
    """ace_eval_grad folds conjugate pairs on the remat and forest schedules;
    the flag ACE_FLAG_UNFOLDED evaluates every tuple.  Both match, and the oracle."""
    import paper_2202_04140_amd as ace
    print(f"folded wid={wid} n_env={n_env} sched={sched}", flush=True)
    G = graph(wid, device, sched)
    g, K, c = oracle_basis(wid)
    off, pos = problem(wid, n_env)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi_f, grad_f = ace.eval_grad(G, tc, toff, tpos)
    phi_u, grad_u = ace.eval_grad(G, tc, toff, tpos, unfolded=True)
    assert rel(cplx(phi_f), cplx(phi_u)) <= TOL_PHI
    assert rel(grad_f.cpu().numpy(), grad_u.cpu().numpy()) <= TOL_GRAD
    phi_e = ace.eval(G, tc, toff, tpos)
    assert rel(cplx(phi_e), cplx(phi_u)) <= TOL_PHI
    if wid in (3, 4):
        phi_ref, g_ref = oc.grad_naive(g.labels, K, c, off, pos, wl.WORKLOADS[wid].r_cut)
        assert rel(cplx(phi_f), phi_ref) <= TOL_PHI
        assert rel(grad_f.cpu().numpy(), g_ref) <= TOL_GRAD


@pytest.mark.parametrize("wid,n_env", [(2, 32), (4, 8)])
def test_contract_conj_symmetric_folds(device, wid, n_env):
    """ace_contract with ACE_FLAG_CONJ_SYMMETRIC on conjugate-symmetric A: phi as
    the oracle's, and Abar gives the oracle's d Re(phi) along symmetric directions."""
    import paper_2202_04140_amd as ace
    print(f"contract conj wid={wid} n_env={n_env}", flush=True)
    for sched in ("remat", None):
        G = graph(wid, device, sched)
        g, K, c = oracle_basis(wid)
        A = wl.random_A_conj(n_env, g.labels, 200 + wid) * 0.5
        dA = wl.random_A_conj(n_env, g.labels, 300 + wid)
        tc, tA = to_dev(device, c, np.stack([A.real, A.imag], -1))
        phi, Ab = ace.contract(G, tc, tA, with_grad=True, conj_symmetric=True)
        phi_ref = oc.phi_naive(K, c, A)
        ab_ref = oc.abar_naive(K, c, A)
        assert rel(cplx(phi), phi_ref) <= TOL_PHI
        lhs = np.real(np.sum(cplx(Ab) * dA, axis=1))
        rhs = np.real(np.sum(ab_ref * dA, axis=1))
        assert rel(lhs, rhs) <= TOL_ABAR


# ---- Algorithm 2 and p-norm degree sets (Sec. 2.5, Sec. 3.3) ---------------------------
F1_SPECS = [dict(nu=4, D=8, nl=4, alg=2, n=2, p=1), dict(nu=3, D=6, nl=3, alg=1, n=1, p=2),
            dict(nu=4, D=6, nl=3, alg=2, n=2, p=2), dict(nu=3, D=5, nl=3, alg=2, n=2, p=math.inf)]


@pytest.mark.parametrize("sched", [None, "remat"])
@pytest.mark.parametrize("k", range(len(F1_SPECS)))
def test_alg2_and_p_norm_graphs_eval_grad(device, k, sched):
    import paper_2202_04140_amd as ace
    sp = F1_SPECS[k]
    print(f"f1 spec={sp} sched={sched}", flush=True)
    G = ace.Graph(sp["nu"], sp["D"], sp["nl"], sp["nl"], algorithm=sp["alg"], alg_n=sp["n"], degree_p=sp["p"])
    if sched:
        G.set_schedule(schedule=sched)
    g = group_o3(sp["nl"], sp["nl"], sp["D"])
    K = all_invariant_tuples(g, sp["nu"], sp["D"], sp["p"])
    kt = G.k_tuples()
    assert [tuple(x for x in row if x >= 0) for row in kt] == K
    c = np.random.default_rng(40 + k).standard_normal(len(K)) / (1.0 + np.array([g.degree(t) for t in K])) ** 2
    counts = [5, 9, 1, 12, 0, 30]
    off = np.zeros(len(counts) + 1, np.int32)
    off[1:] = np.cumsum(counts)
    pos = wl.positions(int(off[-1]), 90 + k)
    tc, toff, tpos = to_dev(device, c, off, pos)
    phi, grad = ace.eval_grad(G, tc, toff, tpos)
    phi_ref, g_ref = oc.grad_naive(g.labels, K, c, off, pos, 5.0)
    assert rel(cplx(phi), phi_ref) <= TOL_PHI
    assert rel(grad.cpu().numpy(), g_ref) <= TOL_GRAD
    phi_n, grad_n = ace.eval_grad(G, tc, toff, tpos, naive=True)
    assert rel(cplx(phi_n), phi_ref) <= TOL_PHI
