"""hipGraph capture of the whole step, and schedule variants, on the GPU."""

import numpy as np
import pytest

import workloads as wl
from oracle import contraction as oc
from oracle.indexsets import all_invariant_tuples, group_o3

pytestmark = pytest.mark.gpu


def setup(device, wid=3, n_env=256):
    import torch
    import paper_2202_04140_amd as ace
    w = wl.WORKLOADS[wid]
    G = ace.Graph(w.nu_max, w.degree_max, w.n_max, w.l_max, r_cut=w.r_cut)
    off, pos = wl.batch(w)
    off, pos = wl.gather(off, pos, wl.subset(off, n_env))
    c = wl.coefficients(w, G.k_degrees())
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return ace, G, t(c), t(off), t(pos), off, pos


def rel(a, b):
    import torch
    return (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()


def test_graph_capture_replays_match_eager(device):
    import torch
    print("graph capture wid=3 n_env=256", flush=True)
    ace, G, tc, toff, tpos, off, pos = setup(device)
    phi_e, grad_e = ace.eval_grad(G, tc, toff, tpos)
    phi = torch.empty_like(phi_e)
    grad = torch.empty_like(grad_e)
    ace.eval_grad(G, tc, toff, tpos, out=(phi, grad))     # warm-up before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ace.eval_grad(G, tc, toff, tpos, out=(phi, grad))
    torch.cuda.synchronize()
    other = torch.from_numpy(wl.positions(pos.shape[0], 55)).to(device)
    for r in range(4):
        # eager work and synchronisation between replays
        ace.eval(G, tc, toff, other)
        phi.zero_()
        grad.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert rel(phi, phi_e) <= 1e-13, r
        assert rel(grad, grad_e) <= 1e-12, r


def test_graph_replay_follows_new_inputs(device):
    """Replays read the captured input buffers: new positions copied into them give new results."""
    import torch
    ace, G, tc, toff, tpos, off, pos = setup(device, n_env=64)
    buf = tpos.clone()
    phi = torch.empty((64, 2), dtype=torch.float64, device=device)
    grad = torch.empty_like(buf)
    ace.eval_grad(G, tc, toff, buf, out=(phi, grad))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ace.eval_grad(G, tc, toff, buf, out=(phi, grad))
    for seed in (56, 57):
        new = torch.from_numpy(wl.positions(buf.shape[0], seed)).to(device)
        buf.copy_(new)
        g.replay()
        torch.cuda.synchronize()
        ref_phi, ref_grad = ace.eval_grad(G, tc, toff, new)
        assert rel(phi, ref_phi) <= 1e-13
        assert rel(grad, ref_grad) <= 1e-12


@pytest.mark.parametrize("opts", [dict(row_chunk=8, tree_chunk=2, hot_columns=0, bank_schedule=0, block_threads=256),
                                  dict(row_chunk=64, tree_chunk=32, hot_columns=2, bank_schedule=1, block_threads=128),
                                  dict(schedule="remat", term_chunk=3, pair_slots=0, bank_schedule=0, hot_columns=0,
                                       block_threads=64),
                                  dict(schedule="remat", term_chunk=64, pair_slots=4096, bank_schedule=1,
                                       hot_columns=4, block_threads=512)])
def test_schedule_variants_keep_parity(device, opts):
    print(f"schedule {opts}", flush=True)
    import torch
    import paper_2202_04140_amd as ace
    w = wl.WORKLOADS[2]
    G = ace.Graph(w.nu_max, w.degree_max, w.n_max, w.l_max, r_cut=w.r_cut)
    G.set_schedule(**opts)
    got = G.get_schedule()
    assert {k: got[k] for k in opts} == opts
    g = group_o3(w.n_max, w.l_max, w.degree_max)
    K = all_invariant_tuples(g, w.nu_max, w.degree_max)
    c = wl.coefficients(w, np.array([g.degree(k) for k in K]))
    A = wl.random_A(24, len(g), 77) * 0.5
    tA = torch.from_numpy(np.stack([A.real, A.imag], -1)).to(device)
    phi, Ab = ace.contract(G, torch.from_numpy(c).to(device), tA, with_grad=True)
    phi = phi.cpu().numpy()
    Ab = Ab.cpu().numpy()
    pr, ar = oc.phi_naive(K, c, A), oc.abar_naive(K, c, A)
    assert np.linalg.norm(phi[:, 0] + 1j * phi[:, 1] - pr) <= 1e-11 * np.linalg.norm(pr)
    assert np.linalg.norm(Ab[..., 0] + 1j * Ab[..., 1] - ar) <= 1e-11 * np.linalg.norm(ar)


def test_autotuner_applies_a_valid_schedule(device, tmp_path, monkeypatch):
    import paper_2202_04140_amd as ace
    from paper_2202_04140_amd import autotune
    monkeypatch.setenv("ACE_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    ace_, G, tc, toff, tpos, off, pos = setup(device, n_env=128)
    A = ace.basis(G, toff, tpos)
    ref_phi, _ = ace.eval_grad(G, tc, toff, tpos)
    res = autotune.tune(G, tc, A, reps=2)
    assert not res["cached"] and len(res["tried"]) > 3
    assert G.get_schedule() == res["opts"]
    phi, _ = ace.eval_grad(G, tc, toff, tpos)
    assert rel(phi, ref_phi) <= 1e-13
    res2 = autotune.tune(G, tc, A, reps=2)
    assert res2["cached"] and res2["opts"] == res["opts"]
