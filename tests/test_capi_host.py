"""Host-side tests of libace.so: exports, the graph builder (bit-exact
against the oracle builder), statistics and error handling.  No GPU needed."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2202_04140_amd as ace
from oracle.graph import OracleGraph
from oracle.indexsets import group_o3, group_torus

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "ace.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ace_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ace.lib()
    names = header_functions()
    assert "ace_eval_grad" in names and "ace_graph_build" in names
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a prototype for each of them
    assert set(names) == set(ace.EXPORTED)


def test_version_and_no_error():
    assert ace.lib().ace_version().startswith(b"ace-dag")


def oracle_arrays(group, nu, D, alg=1, n=1, p=1):
    G = OracleGraph(group, nu, D, alg, n, p=p)
    tup = np.full((G.n_nodes(), nu), -1, np.int32)
    for v, t in enumerate(G.node_tuple):
        tup[v, :len(t)] = t
    par = np.array([p if p is not None else (-1, -1) for p in G.parents], np.int32)
    return G, tup, par, np.array(G.k_to_node, np.int64)


@pytest.mark.parametrize("spec,alg,n", [((4, 4, 8, 3), 1, 1), ((6, 6, 12, 4), 1, 1),
                                        ((4, 4, 8, 3), 2, 2), ((6, 6, 12, 4), 2, 2),
                                        ((3, 2, 9, 5), 1, 1), ((2, 3, 10, 6), 2, 3)])
def test_builder_bit_exact_o3(spec, alg, n):
    nmax, lmax, D, nu = spec
    g = ace.Graph(nu, D, nmax, lmax, algorithm=alg, alg_n=n, host_only=True)
    onep, tup, par, k2n = g.export()
    G, otup, opar, ok2n = oracle_arrays(group_o3(nmax, lmax, D), nu, D, alg, n)
    assert onep.tolist() == [list(t) for t in G.group.labels]
    np.testing.assert_array_equal(tup, otup)
    np.testing.assert_array_equal(par, opar)
    np.testing.assert_array_equal(k2n, ok2n)
    kt = g.k_tuples()
    okt = np.full((len(G.K), nu), -1, np.int32)
    for q, k in enumerate(G.K):
        okt[q, :len(k)] = k
    np.testing.assert_array_equal(kt, okt)
    st = g.stats()
    assert st["n_aux"] == G.aux_count()
    lay = G.layers()
    assert st["depth"] == max(lay)
    assert st["n_layer"][:max(lay) + 1] == [lay.count(L) for L in range(max(lay) + 1)]


@pytest.mark.parametrize("p", [2, math.inf])
@pytest.mark.parametrize("spec,alg,n", [((3, 3, 6, 3), 1, 1), ((3, 3, 6, 4), 1, 1), ((3, 3, 6, 4), 2, 2),
                                        ((2, 2, 5, 5), 2, 3)])
def test_builder_bit_exact_o3_p_norm(spec, alg, n, p):
    nmax, lmax, D, nu = spec
    g = ace.Graph(nu, D, nmax, lmax, algorithm=alg, alg_n=n, degree_p=p, host_only=True)
    onep, tup, par, k2n = g.export()
    G, otup, opar, ok2n = oracle_arrays(group_o3(nmax, lmax, D), nu, D, alg, n, p)
    assert onep.tolist() == [list(t) for t in G.group.labels]
    np.testing.assert_array_equal(tup, otup)
    np.testing.assert_array_equal(par, opar)
    np.testing.assert_array_equal(k2n, ok2n)
    assert g.stats()["n_aux"] == G.aux_count()


@pytest.mark.parametrize("p", [2, math.inf])
def test_builder_bit_exact_torus_p_norm(p):
    for nu, D, alg, n in [(4, 8, 1, 1), (5, 8, 2, 2)]:
        g = ace.Graph(nu, D, group=ace.GROUP_TORUS, algorithm=alg, alg_n=n, degree_p=p, host_only=True)
        _, tup, par, k2n = g.export()
        _, otup, opar, ok2n = oracle_arrays(group_torus(D), nu, D, alg, n, p)
        np.testing.assert_array_equal(tup, otup)
        np.testing.assert_array_equal(par, opar)
        np.testing.assert_array_equal(k2n, ok2n)


def test_invalid_degree_p():
    with pytest.raises(ValueError):
        ace.Graph(3, 6, 2, 2, degree_p=3, host_only=True)
    spec = ace._Spec(group=0, nu_max=3, degree_max=6, n_max=2, l_max=2, algorithm=1, alg_n=1, degree_p=5,
                     r_cut=5.0, build_flags=1, reserved2=0)
    h = ctypes.c_void_p()
    assert ace.lib().ace_graph_build(ctypes.byref(spec), ctypes.byref(h)) == 1
    assert b"degree_p" in ace.lib().ace_last_error()


@pytest.mark.parametrize("nu,D,alg,n", [(4, 10, 1, 1), (6, 12, 1, 1), (5, 12, 2, 2)])
def test_builder_bit_exact_torus(nu, D, alg, n):
    g = ace.Graph(nu, D, group=ace.GROUP_TORUS, algorithm=alg, alg_n=n, host_only=True)
    _, tup, par, k2n = g.export()
    _, otup, opar, ok2n = oracle_arrays(group_torus(D), nu, D, alg, n)
    np.testing.assert_array_equal(tup, otup)
    np.testing.assert_array_equal(par, opar)
    np.testing.assert_array_equal(k2n, ok2n)


@pytest.mark.parametrize("alg,n", [(1, 1), (2, 2), (2, 3)])
def test_builder_matches_hand_worked_torus_graph(alg, n):
    """The library builder against the node lists worked by hand for the
    torus, nu <= 4, D = 6 (tests/golden/alg2_torus_nu4_D6.txt)."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_oracle_graph import _hand_worked_lists
    expected = _hand_worked_lists()[(alg, n)]
    g = ace.Graph(4, 6, group=ace.GROUP_TORUS, algorithm=alg, alg_n=n, host_only=True)
    _, tup, par, _ = g.export()
    assert tup.shape[0] == 13 + len(expected)
    for v, t, pr in expected:
        assert tuple(x for x in tup[v] if x >= 0) == t
        assert tuple(par[v]) == pr


# Regression values: |K| per order, V, aux per order, depth, layer sizes, stored and
# childless product nodes, leaves with children, naive complex products.  Every row
# equals the oracle builder's own statistics (test_builder_bit_exact_large for the
# third; the first two come out of the bit-exact tests above).
REGRESSION = {
    (4, 4, 8, 3): dict(k=[15, 228, 959], V=1440, aux=[128], depth=2, layers=[125, 356, 959],
                       S=356, T=959, leafpar=93, naive=2146),
    (6, 6, 12, 4): dict(k=[28, 1098, 9932, 34918], V=47830, aux=[1058, 481], depth=3,
                        layers=[343, 2156, 30381, 14950], S=7511, T=39976, leafpar=263, naive=125716),
    (8, 8, 14, 5): dict(k=[43, 2338, 27320, 122061, 297008], V=453816, aux=[2450, 1585, 374], depth=4,
                        layers=[680, 4788, 97494, 342789, 8065], S=60743, T=392393, leafpar=461,
                        naive=1611193),
}


@pytest.mark.parametrize("spec", list(REGRESSION))
def test_builder_regression_counts(spec):
    nmax, lmax, D, nu = spec
    r = REGRESSION[spec]
    st = ace.Graph(nu, D, nmax, lmax, host_only=True).stats()
    assert st["n_k_by_order"][1:nu + 1] == r["k"]
    assert st["n_nodes"] == r["V"]
    assert st["n_aux_by_order"][2:2 + len(r["aux"])] == r["aux"]
    assert st["depth"] == r["depth"]
    assert st["n_layer"][:r["depth"] + 1] == r["layers"]
    assert st["n_stored"] == r["S"] and st["n_childless"] == r["T"]
    assert st["n_leaf_parents"] == r["leafpar"]
    assert st["naive_cmuls"] == r["naive"]


def oracle_stats(G: OracleGraph, P: int) -> dict:
    """The regression statistics computed from the oracle builder's own DAG."""
    nu = G.nu_max
    lay = G.layers()
    ch = G.child_counts()
    V = G.n_nodes()
    k_by = [0] * (nu + 1)
    for k in G.K:
        k_by[len(k)] += 1
    aux_by = [0] * (nu + 1)
    for v in range(P, V):
        if G.is_aux(v):
            aux_by[len(G.node_tuple[v])] += 1
    depth = max(lay)
    return dict(k=k_by[1:], V=V, aux=[a for a in aux_by[2:] if a] or [], depth=depth,
                layers=[sum(1 for x in lay if x == L) for L in range(depth + 1)],
                S=sum(1 for v in range(P, V) if ch[v] > 0), T=sum(1 for v in range(P, V) if ch[v] == 0),
                leafpar=sum(1 for v in range(P) if ch[v] > 0), naive=sum(len(k) - 1 for k in G.K))


@pytest.mark.parametrize("spec", [pytest.param((8, 8, 14, 5), id="32768-env-basis"),
                                  pytest.param((10, 10, 16, 6), id="8192-env-basis", marks=pytest.mark.slow)])
def test_builder_bit_exact_large(spec):
    """The library builder against the oracle builder on the nu <= 5 and nu <= 6
    bases of the two largest workloads: node lists, parents and K map bit-exact,
    and the stored regression counts equal to the oracle DAG's own statistics."""
    nmax, lmax, D, nu = spec
    g = ace.Graph(nu, D, nmax, lmax, host_only=True)
    onep, tup, par, k2n = g.export()
    grp = group_o3(nmax, lmax, D)
    G = OracleGraph(grp, nu, D, 1, 1)
    V = G.n_nodes()
    assert tup.shape == (V, nu)
    otup = np.full((V, nu), -1, np.int32)
    for v, t in enumerate(G.node_tuple):
        otup[v, :len(t)] = t
    np.testing.assert_array_equal(tup, otup)
    opar = np.array([p if p is not None else (-1, -1) for p in G.parents], np.int32)
    np.testing.assert_array_equal(par, opar)
    np.testing.assert_array_equal(k2n, np.array(G.k_to_node, np.int64))
    ost = oracle_stats(G, len(grp))
    if spec in REGRESSION:
        assert ost == REGRESSION[spec]
    else:
        assert sum(ost["k"]) == 3692953 and ost["V"] == 3705306
        assert ost["aux"] == [4944, 4641, 1373, 314]
        assert ost["S"] == 256091 and ost["T"] == 3448074


def test_torus_theorem_count_through_the_c_builder():
    from oracle.indexsets import torus_aux_count_theorem
    for nu in range(3, 7):
        for D in (4, 8, 12, 20):
            st = ace.Graph(nu, D, group=ace.GROUP_TORUS, host_only=True).stats()
            assert st["n_aux"] == torus_aux_count_theorem(nu, D)


# ---- error paths -----------------------------------------------------------------
@pytest.mark.parametrize("kw", [dict(nu_max=0, degree_max=4), dict(nu_max=9, degree_max=4),
                                dict(nu_max=3, degree_max=-1), dict(nu_max=3, degree_max=4, l_max=17),
                                dict(nu_max=3, degree_max=4, algorithm=3),
                                dict(nu_max=3, degree_max=4, algorithm=2, alg_n=0),
                                dict(nu_max=3, degree_max=4, r_cut=0.0),
                                dict(nu_max=3, degree_max=4, group=7)])
def test_invalid_spec(kw):
    with pytest.raises(ace.AceError) as ei:
        ace.Graph(host_only=True, **kw)
    assert ei.value.status == 1
    assert len(ace.lib().ace_last_error()) > 0


def test_null_arguments():
    lib = ace.lib()
    assert lib.ace_graph_build(None, None) == 1
    assert lib.ace_graph_info(None, None) == 1
    assert lib.ace_graph_export(None, None, None, None, None) == 1
    out = ctypes.c_size_t()
    assert lib.ace_workspace_size(None, 1, 1, 0, ctypes.byref(out)) == 1
    lib.ace_graph_free(None)  # no-op


def test_host_only_graph_rejects_device_calls():
    g = ace.Graph(3, 8, 4, 4, host_only=True)
    lib = ace.lib()
    out = ctypes.c_size_t()
    assert lib.ace_workspace_size(g.handle, 4, 4, 0, ctypes.byref(out)) == 1
    assert lib.ace_eval(g.handle, None, 1, None, None, None, None, 0, 0, None) == 1
    assert b"HOST_ONLY" in lib.ace_last_error()


def test_device_build_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(ace.AceError) as ei:
        ace.Graph(3, 8, 4, 4)
    assert ei.value.status == 4


# ---- forest schedule: host emulation of the kernel's exact index logic ------------
@pytest.mark.parametrize("spec,n_env", [((4, 4, 8, 3), 4), ((6, 6, 12, 4), 3), ((8, 8, 14, 5), 2),
                                        ((3, 2, 9, 5), 3)])
def test_forest_schedule_host_emulation_matches_oracle(spec, n_env):
    from oracle import contraction as oc
    from oracle.indexsets import all_invariant_tuples
    import workloads as wl
    nmax, lmax, D, nu = spec
    G = ace.Graph(nu, D, nmax, lmax, host_only=True)
    if G.schedule_kind() != "forest":
        pytest.skip("graph uses the layered schedule")
    g = group_o3(nmax, lmax, D)
    K = all_invariant_tuples(g, nu, D)
    rng = np.random.default_rng(9)
    c = rng.standard_normal(len(K))
    A = wl.random_A(n_env, len(g), 21) * 0.5
    phi, ab = G.forest_eval_host(c, A)
    pr, ar = oc.phi_naive(K, c, A), oc.abar_naive(K, c, A)
    assert np.linalg.norm(phi - pr) <= 1e-13 * np.linalg.norm(pr)
    assert np.linalg.norm(ab - ar) <= 1e-13 * np.linalg.norm(ar)


def test_schedule_kinds():
    assert ace.Graph(3, 8, 4, 4, host_only=True).schedule_kind() == "forest"
    assert ace.Graph(4, 12, 6, 6, host_only=True).schedule_kind() == "forest"
    # order-6 products of two order-3 nodes have no resident parent: the
    # forest does not apply and the remat schedule takes over
    g = ace.Graph(6, 10, 3, 3, host_only=True)
    assert g.schedule_kind() == "remat"
    with pytest.raises(ace.AceError) as ei:
        g.set_schedule(schedule="forest")
    assert ei.value.status == 2 and b"two non-resident parents" in ace.lib().ace_last_error()
    g.set_schedule(schedule="layered")
    assert g.schedule_kind() == "layered"
    g2 = ace.Graph(3, 8, 4, 4, host_only=True)
    g2.set_schedule(schedule="remat", term_chunk=3)
    assert g2.schedule_kind() == "remat" and g2.get_schedule()["term_chunk"] == 3
    for bad in (dict(term_chunk=0), dict(term_chunk=257), dict(schedule=4), dict(env_per_block=0),
                dict(env_per_block=3)):
        with pytest.raises(ace.AceError):
            g2.set_schedule(**bad)


def test_failed_set_schedule_leaves_every_option_and_layout_unchanged():
    """A set_schedule call that fails (here: a forest on a graph that has none)
    must leave the options and the schedules as they were, including the
    options it would have changed along the way."""
    from oracle import contraction as oc
    from oracle.indexsets import all_invariant_tuples
    import workloads as wl
    g = ace.Graph(6, 6, 2, 2, host_only=True)
    g.set_schedule(schedule="remat", term_chunk=64, pair_slots=100, hot_columns=2)
    before = (g.get_schedule(), g.schedule_info())
    with pytest.raises(ace.AceError) as ei:
        g.set_schedule(schedule="forest", term_chunk=16, pair_slots=0, hot_columns=4, row_chunk=8)
    assert ei.value.status == 2
    assert (g.get_schedule(), g.schedule_info()) == before
    gr = group_o3(2, 2, 6)
    K = all_invariant_tuples(gr, 6, 6)
    c = np.random.default_rng(3).standard_normal(len(K))
    A = wl.random_A(2, len(gr), 5) * 0.5
    phi, ab = g.remat_eval_host(c, A)
    pr, ar = oc.phi_naive(K, c, A), oc.abar_naive(K, c, A)
    assert np.linalg.norm(phi - pr) <= 1e-13 * np.linalg.norm(pr)
    assert np.linalg.norm(ab - ar) <= 1e-13 * np.linalg.norm(ar)
    # an out-of-range option is rejected before anything is touched
    with pytest.raises(ace.AceError):
        g.set_schedule(term_chunk=0)
    assert (g.get_schedule(), g.schedule_info()) == before


# ---- remat schedule: host emulation of the kernel's exact index logic -------------
@pytest.mark.parametrize("spec,alg,n,chunk,pairs", [((4, 4, 8, 3), 1, 1, 16, 0), ((6, 6, 12, 4), 1, 1, 5, 64),
                                                    ((6, 6, 12, 4), 2, 2, 16, 2048), ((3, 2, 9, 5), 1, 1, 1, 7),
                                                    ((2, 2, 10, 6), 1, 1, 7, 30), ((2, 2, 10, 6), 2, 3, 16, 0),
                                                    ((2, 1, 8, 8), 1, 1, 4, 100)])
def test_remat_schedule_host_emulation_matches_oracle(spec, alg, n, chunk, pairs):
    from oracle import contraction as oc
    from oracle.indexsets import all_invariant_tuples
    import workloads as wl
    nmax, lmax, D, nu = spec
    G = ace.Graph(nu, D, nmax, lmax, algorithm=alg, alg_n=n, host_only=True)
    G.set_schedule(schedule="remat", term_chunk=chunk, hot_columns=2, pair_slots=pairs)
    info = G.schedule_info()
    n_terms = G.stats()["n_k"] - G.stats()["n_k_by_order"][1]
    assert info["kind"] == "remat" and info["fwd_entry_real"] == n_terms
    assert n_terms < info["entry_real"] <= 2 * n_terms
    assert info["pairs"] <= pairs
    g = group_o3(nmax, lmax, D)
    K = all_invariant_tuples(g, nu, D)
    c = np.random.default_rng(8).standard_normal(len(K))
    A = wl.random_A(3, len(g), 23) * 0.5
    phi, ab = G.remat_eval_host(c, A)
    pr, ar = oc.phi_naive(K, c, A), oc.abar_naive(K, c, A)
    assert np.linalg.norm(phi - pr) <= 1e-13 * np.linalg.norm(pr)
    assert np.linalg.norm(ab - ar) <= 1e-13 * np.linalg.norm(ar)


# ---- folded remat schedules (conjugate pairs) -------------------------------------
@pytest.mark.parametrize("spec,alg,n", [((4, 4, 8, 3), 1, 1), ((6, 6, 12, 4), 1, 1), ((6, 6, 12, 4), 2, 2),
                                        ((2, 2, 10, 6), 1, 1)])
def test_folded_remat_matches_oracle_for_conjugate_symmetric_A(spec, alg, n):
    """phi from one tuple of each conjugate pair, and Re sum_i Abar'_i dA_i equal to
    the oracle's d Re(phi) for conjugate-symmetric directions dA."""
    from oracle import contraction as oc
    from oracle.indexsets import all_invariant_tuples
    import workloads as wl
    nmax, lmax, D, nu = spec
    G = ace.Graph(nu, D, nmax, lmax, algorithm=alg, alg_n=n, host_only=True)
    G.set_schedule(schedule="remat")
    info = G.schedule_info()
    g = group_o3(nmax, lmax, D)
    K = all_invariant_tuples(g, nu, D)
    # one tuple per conjugate pair (self-conjugate tuples stay)
    n_terms = G.stats()["n_k"] - G.stats()["n_k_by_order"][1]
    assert info["folded_entry_real"] < 0.8 * info["entry_real"]
    c = np.random.default_rng(12).standard_normal(len(K))
    A = wl.random_A_conj(3, g.labels, 31) * 0.5
    dA = wl.random_A_conj(3, g.labels, 32)
    phi, ab = G.remat_eval_host(c, A, folded=True)
    pr, ar = oc.phi_naive(K, c, A), oc.abar_naive(K, c, A)
    assert np.linalg.norm(phi - pr) <= 1e-13 * np.linalg.norm(pr)
    lhs = np.real(np.sum(ab * dA, axis=1))
    rhs = np.real(np.sum(ar * dA, axis=1))
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)
    # for a general A the folded adjoint is not dphi/dA
    assert np.linalg.norm(ab - ar) > 1e-6 * np.linalg.norm(ar)


# ---- folded forest schedule (conjugate pairs) --------------------------------------
@pytest.mark.parametrize("spec,alg,n", [((4, 4, 8, 3), 1, 1), ((6, 6, 12, 4), 1, 1), ((6, 6, 12, 4), 2, 2),
                                        ((3, 2, 9, 5), 1, 1)])
def test_folded_forest_matches_oracle_for_conjugate_symmetric_A(spec, alg, n):
    """The forest over one tuple of each conjugate pair: phi exact for
    conjugate-symmetric A, and Re sum_i Abar'_i dA_i equal to the oracle's
    d Re(phi) along conjugate-symmetric directions dA."""
    from oracle import contraction as oc
    from oracle.indexsets import all_invariant_tuples
    import workloads as wl
    nmax, lmax, D, nu = spec
    G = ace.Graph(nu, D, nmax, lmax, algorithm=alg, alg_n=n, host_only=True)
    if G.schedule_kind() != "forest":
        pytest.skip("graph uses another schedule")
    info = G.schedule_info()
    assert 0 < info["folded_real"] < 0.9 * (info["child_real"] + info["entry_real"])
    g = group_o3(nmax, lmax, D)
    K = all_invariant_tuples(g, nu, D)
    c = np.random.default_rng(13).standard_normal(len(K))
    A = wl.random_A_conj(3, g.labels, 33) * 0.5
    dA = wl.random_A_conj(3, g.labels, 34)
    phi, ab = G.forest_eval_host(c, A, folded=True)
    pr, ar = oc.phi_naive(K, c, A), oc.abar_naive(K, c, A)
    assert np.linalg.norm(phi - pr) <= 1e-13 * np.linalg.norm(pr)
    lhs = np.real(np.sum(ab * dA, axis=1))
    rhs = np.real(np.sum(ar * dA, axis=1))
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)
    assert np.linalg.norm(ab - ar) > 1e-6 * np.linalg.norm(ar)
    # the unfolded forest is exact for any A
    A2 = wl.random_A(2, len(g), 35) * 0.5
    phi2, ab2 = G.forest_eval_host(c, A2, folded=False)
    assert np.linalg.norm(phi2 - oc.phi_naive(K, c, A2)) <= 1e-13 * np.linalg.norm(phi2)
    assert np.linalg.norm(ab2 - oc.abar_naive(K, c, A2)) <= 1e-13 * np.linalg.norm(ab2)


@pytest.mark.parametrize("group", ["so2", "torus", "features"])
def test_folded_forest_other_groups_matches_oracle(group):
    """Folded forest on pooled one-particle values of the planar groups and of
    an O(3) basis with an invariant feature."""
    from oracle import contraction as oc
    from oracle import onebody as ob
    from oracle.indexsets import all_invariant_tuples, group_o3_features, group_so2
    import workloads as wl
    if group == "so2":
        G = ace.Graph(4, 8, 4, 4, group=ace.GROUP_SO2, host_only=True)
        g = group_so2(4, 4, 8)
        K = all_invariant_tuples(g, 4, 8)
        off = np.array([0, 6, 13, 20], np.int32)
        pos = wl.planar_positions(20, 6, circle=False)
    elif group == "torus":
        G = ace.Graph(5, 8, group=ace.GROUP_TORUS, host_only=True)
        g = group_torus(8)
        K = all_invariant_tuples(g, 5, 8)
        off = np.array([0, 6, 13, 20], np.int32)
        pos = wl.planar_positions(20, 7, circle=True)
    else:
        G = ace.Graph(4, 8, 3, 3, k_max=2, host_only=True)
        g = group_o3_features(3, 3, 2, 8)
        K = all_invariant_tuples(g, 4, 8)
        rng = np.random.default_rng(3)
        d = rng.standard_normal((15, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        pos = np.concatenate([d * rng.uniform(0.5, 5, 15)[:, None], rng.uniform(-1, 1, (15, 1))], axis=1)
        off = np.array([0, 7, 15], np.int32)
    if G.schedule_kind() != "forest":
        pytest.skip("graph uses another schedule")
    c = np.random.default_rng(4).standard_normal(len(K))
    A = ob.pooled_A(g.labels, off, pos, 5.0)
    pr = oc.phi_naive(K, c, A)
    for folded in (False, True):
        phi, _ = G.forest_eval_host(c, A, folded=folded)
        assert np.linalg.norm(phi - pr) <= 1e-13 * np.linalg.norm(pr)


# ---- planar groups: SO(2) builder and schedules ------------------------------------
@pytest.mark.parametrize("spec,alg,n", [((3, 3, 6, 4), 1, 1), ((4, 4, 8, 3), 2, 2), ((2, 5, 7, 5), 1, 1)])
def test_builder_bit_exact_so2(spec, alg, n):
    from oracle.indexsets import group_so2
    nmax, mmax, D, nu = spec
    g = ace.Graph(nu, D, nmax, mmax, group=ace.GROUP_SO2, algorithm=alg, alg_n=n, host_only=True)
    onep, tup, par, k2n = g.export()
    G, otup, opar, ok2n = oracle_arrays(group_so2(nmax, mmax, D), nu, D, alg, n)
    assert [(int(a), int(c)) for a, _, c in onep] == G.group.labels
    np.testing.assert_array_equal(tup, otup)
    np.testing.assert_array_equal(par, opar)
    np.testing.assert_array_equal(k2n, ok2n)


@pytest.mark.parametrize("group", ["so2", "torus"])
def test_folded_remat_planar_matches_oracle(group):
    """Folded remat schedules on pooled planar one-particle values (which satisfy
    A_{n,-m} = conj(A_{n,m})) against the oracle."""
    from oracle import contraction as oc
    from oracle import onebody as ob
    from oracle.indexsets import all_invariant_tuples, group_so2
    import workloads as wl
    if group == "so2":
        G = ace.Graph(4, 8, 4, 4, group=ace.GROUP_SO2, host_only=True)
        g = group_so2(4, 4, 8)
        K = all_invariant_tuples(g, 4, 8)
    else:
        G = ace.Graph(5, 8, group=ace.GROUP_TORUS, host_only=True)
        g = group_torus(8)
        K = all_invariant_tuples(g, 5, 8)
    G.set_schedule(schedule="remat")
    c = np.random.default_rng(4).standard_normal(len(K))
    off = np.array([0, 6, 13, 20], np.int32)
    pos = wl.planar_positions(20, 6, circle=group == "torus")
    A = ob.pooled_A(g.labels, off, pos, 5.0)
    for folded in (False, True):
        phi, ab = G.remat_eval_host(c, A, folded=folded)
        pr = oc.phi_naive(K, c, A)
        assert np.linalg.norm(phi - pr) <= 1e-13 * np.linalg.norm(pr)


# ---- invariant features (Sec. 5.4) ---------------------------------------------------
@pytest.mark.parametrize("spec,kmax,alg,n", [((3, 3, 7, 3), 2, 1, 1), ((2, 2, 6, 4), 3, 2, 2)])
def test_builder_bit_exact_features(spec, kmax, alg, n):
    from oracle.indexsets import group_o3_features
    nmax, lmax, D, nu = spec
    g = ace.Graph(nu, D, nmax, lmax, k_max=kmax, algorithm=alg, alg_n=n, host_only=True)
    onep, tup, par, k2n = g.export()
    G, otup, opar, ok2n = oracle_arrays(group_o3_features(nmax, lmax, kmax, D), nu, D, alg, n)
    assert [(int(a), int(b), int(c), int(k)) for (a, b, c), k in zip(onep, g.onep_feature())] == G.group.labels
    np.testing.assert_array_equal(tup, otup)
    np.testing.assert_array_equal(par, opar)
    np.testing.assert_array_equal(k2n, ok2n)
    assert np.array_equal(g.k_degrees(), [G.group.degree(k) for k in G.K])


def test_features_invalid_and_remat_folded():
    from oracle import contraction as oc
    from oracle import onebody as ob
    from oracle.indexsets import all_invariant_tuples, group_o3_features
    with pytest.raises(ace.AceError):
        ace.Graph(3, 6, 2, 2, k_max=17, host_only=True)
    with pytest.raises(ace.AceError):
        ace.Graph(3, 6, 2, 2, group=ace.GROUP_SO2, k_max=1, host_only=True)
    G = ace.Graph(4, 8, 3, 3, k_max=2, host_only=True)
    G.set_schedule(schedule="remat")
    g = group_o3_features(3, 3, 2, 8)
    K = all_invariant_tuples(g, 4, 8)
    c = np.random.default_rng(2).standard_normal(len(K))
    rng = np.random.default_rng(3)
    d = rng.standard_normal((15, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pos = np.concatenate([d * rng.uniform(0.5, 5, 15)[:, None], rng.uniform(-1, 1, (15, 1))], axis=1)
    A = ob.pooled_A(g.labels, np.array([0, 7, 15]), pos, 5.0)
    for folded in (False, True):
        phi, _ = G.remat_eval_host(c, A, folded=folded)
        pr = oc.phi_naive(K, c, A)
        assert np.linalg.norm(phi - pr) <= 1e-13 * np.linalg.norm(pr)


# ---- Sec. 3.4 numerical tests regenerated with the library builder -------------------
def test_aux_ratio_trends_of_sec_3_4():
    """The trends the paper reports for #A/#V: torus, nu = 3: both heuristics insert
    the same auxiliary nodes; nu = 4, 5 at larger D: Algorithm 2 (n = 2) inserts
    fewer.  O(3): for p = 1 Algorithm 2 is slightly worse pre-asymptotically, for
    p = 2 and p = infinity it inserts fewer."""
    import math
    from paper_2202_04140_amd import counts
    for D in (8, 16, 24):
        r = counts.sizes(ace.GROUP_TORUS, 3, D, 1, 1), counts.sizes(ace.GROUP_TORUS, 3, D, 1, 2)
        assert r[0] == r[1]
    for nu in (4, 5):
        a1, a2 = counts.sizes(ace.GROUP_TORUS, nu, 32, 1, 1), counts.sizes(ace.GROUP_TORUS, nu, 32, 1, 2)
        assert a1["K"] == a2["K"] and a2["A"] < a1["A"]
    a1, a2 = counts.sizes(ace.GROUP_O3, 4, 10, 1, 1), counts.sizes(ace.GROUP_O3, 4, 10, 1, 2)
    assert a2["A"] > a1["A"]
    a1, a2 = counts.sizes(ace.GROUP_O3, 4, 8, 2, 1), counts.sizes(ace.GROUP_O3, 4, 8, 2, 2)
    assert a2["A"] < a1["A"]
    a1, a2 = counts.sizes(ace.GROUP_O3, 3, 6, math.inf, 1), counts.sizes(ace.GROUP_O3, 3, 6, math.inf, 2)
    assert a2["A"] < a1["A"]
    rows = counts.table(ace.GROUP_TORUS, 1, [4], [8, 12])
    assert [r[:2] for r in rows] == [(4, 8), (4, 12)] and all(0 < r[5] < 1 for r in rows)


def test_remat_lds_bank_statistics():
    """The remat schedule's LDS statistics follow the bank rules measured on
    gfx950: a quarter-wave of 16-byte reads costs max(2, m) cycles (so the
    mean is at least 2000 x1000), a push instruction puts at least one lane
    on its busiest bank pair, and ordering the entry columns by bank group
    lowers the read cost against the plain order."""
    g = ace.Graph(4, 10, 4, 4, host_only=True)
    cost = {}
    for bs in (1, 0):
        g.set_schedule(schedule="remat", bank_schedule=bs, env_per_block=2, block_threads=1024, hot_columns=2,
                       term_chunk=16)
        info = g.schedule_info()
        assert info["kind"] == "remat"
        assert info["bank_cost_x1000"] >= 2000
        assert 1000 <= info["push_bank_load_x1000"] <= 16000
        cost[bs] = info["bank_cost_x1000"]
    assert cost[1] < cost[0]
