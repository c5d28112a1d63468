"""GPU parity with one invariant feature per neighbour (Sec. 5.4):
phi_nlmk = R_n Y_l^m T_k(mu), positions [N, 4] = (x, y, z, mu)."""

import numpy as np
import pytest

import workloads as wl
from oracle import contraction as oc
from oracle import onebody as ob
from oracle.indexsets import all_invariant_tuples, group_o3_features

pytestmark = pytest.mark.gpu

TOL_A, TOL_PHI, TOL_GRAD = 1e-13, 1e-11, 1e-9


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def cplx(t):
    a = t.detach().cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def setup(n_env, schedule=None):
    import paper_2202_04140_amd as ace
    w = wl.WORKLOADS[8]
    G = ace.Graph(w.nu_max, w.degree_max, w.n_max, w.l_max, k_max=w.k_max, r_cut=w.r_cut)
    if schedule:
        G.set_schedule(schedule=schedule)
    g = group_o3_features(w.n_max, w.l_max, w.k_max, w.degree_max)
    K = all_invariant_tuples(g, w.nu_max, w.degree_max)
    assert [tuple(x for x in row if x >= 0) for row in G.k_tuples()] == K
    c = wl.coefficients(w, G.k_degrees())
    off, pos = wl.batch(w)
    assert pos.shape[1] == 4 and len(np.unique(pos[:, 3])) == 4 and np.abs(pos[:, 3]).max() == 1.0
    off, pos = wl.gather(off, pos, wl.subset(off, n_env))
    return ace, G, g, K, c, off, pos


def dev(device, *arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in arrs]


def test_feature_basis(device):
    print("feature basis", flush=True)
    ace, G, g, K, c, off, pos = setup(64)
    toff, tpos = dev(device, off, pos)
    A = cplx(ace.basis(G, toff, tpos))
    assert rel(A, ob.pooled_A(g.labels, off, pos, 5.0)) <= TOL_A
    with pytest.raises(ValueError):
        ace.basis(G, toff, tpos[:, :3].contiguous())


@pytest.mark.parametrize("schedule", [None, "remat", "layered"])
def test_feature_eval_grad(device, schedule):
    print(f"feature eval_grad schedule={schedule}", flush=True)
    ace, G, g, K, c, off, pos = setup(40, schedule)
    tc, toff, tpos = dev(device, c, off, pos)
    phi_ref, g_ref = oc.grad_naive(g.labels, K, c, off, pos, 5.0)
    for kw in ({}, {"unfolded": True}, {"naive": True}):
        phi, grad = ace.eval_grad(G, tc, toff, tpos, **kw)
        assert grad.shape == (pos.shape[0], 3)
        assert rel(cplx(phi), phi_ref) <= TOL_PHI, kw
        assert rel(grad.cpu().numpy(), g_ref) <= TOL_GRAD, kw


def test_feature_autograd_and_central_differences(device):
    import torch
    ace, G, g, K, c, off, pos = setup(6)
    tc, toff, tpos = dev(device, c, off, pos)
    p = tpos.clone().requires_grad_(True)
    e = ace.AceEnergy.apply(p, toff, tc, G)
    e.sum().backward()
    assert p.grad.shape == (pos.shape[0], 4) and torch.all(p.grad[:, 3] == 0)
    _, grad = ace.eval_grad(G, tc, toff, tpos)
    assert torch.allclose(p.grad[:, :3], grad, rtol=1e-12, atol=1e-14 * grad.abs().max().item())
    h = 1e-6
    j = 3
    for d in range(3):
        pp, pm = pos.copy(), pos.copy()
        pp[j, d] += h
        pm[j, d] -= h
        env = int(np.searchsorted(off, j, side="right") - 1)
        fp = ace.eval(G, tc, toff, torch.from_numpy(pp).to(device))[env, 0].item()
        fm = ace.eval(G, tc, toff, torch.from_numpy(pm).to(device))[env, 0].item()
        assert abs(grad[j, d].item() - (fp - fm) / (2 * h)) <= 1e-6 * max(1.0, abs(grad[j, d].item()))
