"""Python binding of libace.so: recursive DAG evaluation of sparse symmetric
ACE contractions on MI355X (gfx950), FP64.

The binding only marshals arguments: every step of the evaluation runs in
the HIP kernels behind the C ABI of include/ace.h.  PyTorch supplies device
memory and the current stream.  If the library has not been built this
module raises on first use; there is no CPU fallback.

    g = Graph(nu_max=4, degree_max=12, n_max=6, l_max=6)
    phi = eval(g, coeffs, offsets, pos)                  # [E, 2] (Re, Im)
    phi, grad = eval_grad(g, coeffs, offsets, pos)       # grad [N, 3]
    e = AceEnergy.apply(pos, offsets, coeffs, g)         # Re phi, differentiable
"""

from __future__ import annotations

import ctypes
import math
import os
import threading

import numpy as np

__all__ = [
    "Graph", "basis", "contract", "eval", "eval_grad", "eval_grad_noalloc", "AceEnergy", "AceError",
    "FLAG_NAIVE", "FLAG_CHECK", "FLAG_LAYERED", "FLAG_UNFOLDED", "FLAG_CONJ_SYMMETRIC", "GROUP_O3", "GROUP_TORUS", "GROUP_SO2", "library_path",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libace.so")

GROUP_O3 = 0
GROUP_TORUS = 1
GROUP_SO2 = 2
BUILD_HOST_ONLY = 1
FLAG_NAIVE = 1
FLAG_CHECK = 2
FLAG_LAYERED = 4
FLAG_UNFOLDED = 8
FLAG_CONJ_SYMMETRIC = 16
SCHEDULES = {"auto": 0, "forest": 1, "remat": 2, "layered": 3}
_KIND = {0: "layered", 1: "forest", 2: "remat"}

_STATUS = {0: "ACE_OK", 1: "ACE_ERR_INVALID_ARG", 2: "ACE_ERR_UNSUPPORTED",
           3: "ACE_ERR_OUT_OF_MEMORY", 4: "ACE_ERR_HIP", 5: "ACE_ERR_INTERNAL"}


class AceError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Spec(ctypes.Structure):
    _fields_ = [("group", ctypes.c_int32), ("nu_max", ctypes.c_int32),
                ("degree_max", ctypes.c_int32), ("n_max", ctypes.c_int32),
                ("l_max", ctypes.c_int32), ("algorithm", ctypes.c_int32),
                ("alg_n", ctypes.c_int32), ("degree_p", ctypes.c_int32),
                ("r_cut", ctypes.c_double), ("build_flags", ctypes.c_uint32),
                ("k_max", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("row_chunk", ctypes.c_int32), ("tree_chunk", ctypes.c_int32),
                ("hot_columns", ctypes.c_int32), ("bank_schedule", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("term_chunk", ctypes.c_int32), ("pair_slots", ctypes.c_int32),
                ("env_per_block", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_onep", ctypes.c_int64), ("n_k", ctypes.c_int64),
                ("n_k_by_order", ctypes.c_int64 * 9), ("n_nodes", ctypes.c_int64),
                ("n_aux", ctypes.c_int64), ("n_aux_by_order", ctypes.c_int64 * 9),
                ("depth", ctypes.c_int64), ("n_stored", ctypes.c_int64),
                ("n_childless", ctypes.c_int64), ("n_leaf_parents", ctypes.c_int64),
                ("n_layer", ctypes.c_int64 * 16), ("naive_cmuls", ctypes.c_int64)]


_lib = None
_lib_lock = threading.Lock()

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_SZ = ctypes.c_size_t

EXPORTED = {
    "ace_last_error": ([], ctypes.c_char_p),
    "ace_version": ([], ctypes.c_char_p),
    "ace_graph_build": ([ctypes.POINTER(_Spec), ctypes.POINTER(_P)], ctypes.c_int32),
    "ace_graph_free": ([_P], None),
    "ace_graph_info": ([_P, ctypes.POINTER(_Stats)], ctypes.c_int32),
    "ace_graph_export": ([_P, _P, _P, _P, _P], ctypes.c_int32),
    "ace_graph_export_k": ([_P, _P], ctypes.c_int32),
    "ace_graph_export_feature": ([_P, _P], ctypes.c_int32),
    "ace_workspace_size": ([_P, _I64, _I64, _U32, ctypes.POINTER(_SZ)], ctypes.c_int32),
    "ace_basis": ([_P, _I64, _P, _P, _P, _P], ctypes.c_int32),
    "ace_contract": ([_P, _P, _I64, _P, _P, _P, _P, _SZ, _U32, _P], ctypes.c_int32),
    "ace_eval": ([_P, _P, _I64, _P, _P, _P, _P, _SZ, _U32, _P], ctypes.c_int32),
    "ace_eval_grad": ([_P, _P, _I64, _P, _P, _P, _P, _P, _SZ, _U32, _P], ctypes.c_int32),
    "ace_eval_grad_noalloc": ([_P, _P, _I64, _P, _P, _P, _P, _U32, _P], ctypes.c_int32),
    "ace_check_offsets_result": ([_P], ctypes.c_int32),
    "ace_graph_get_schedule": ([_P, ctypes.POINTER(_Opts)], ctypes.c_int32),
    "ace_graph_set_schedule": ([_P, ctypes.POINTER(_Opts)], ctypes.c_int32),
    "ace_debug_schedule": ([_P, ctypes.POINTER(ctypes.c_int32), _P], ctypes.c_int32),
    "ace_debug_forest_eval": ([_P, _P, _I64, _P, _P, _P, ctypes.c_int32], ctypes.c_int32),
    "ace_debug_remat_eval": ([_P, _P, _I64, _P, _P, _P, ctypes.c_int32], ctypes.c_int32),
}


def library_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded libace.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError(
                    f"{_LIB_PATH} is missing: build it with `python -m paper_2202_04140_amd.build` "
                    "(there is no CPU fallback)")
            handle = ctypes.CDLL(_LIB_PATH)
            for name, (args, res) in EXPORTED.items():
                fn = getattr(handle, name)
                fn.argtypes = args
                fn.restype = res
            _lib = handle
    return _lib


def _check(status: int):
    if status != 0:
        raise AceError(status, lib().ace_last_error().decode())


# ---------------------------------------------------------------------------
class Graph:
    """The DAG for a basis specification (ace_graph_build)."""

    def __init__(self, nu_max: int, degree_max: int, n_max: int = 0, l_max: int = 0, *,
                 group: int = GROUP_O3, algorithm: int = 1, alg_n: int = 1, r_cut: float = 5.0,
                 degree_p=1, k_max: int = 0, host_only: bool = False):
        """degree_p: 1 (total degree), 2 or math.inf: the p-norm of the element
        degrees bounded by degree_max (Sec. 2.5).  k_max > 0: one invariant
        feature per neighbour (Sec. 5.4), positions then [n_nbr, 4] = (x, y, z, mu)."""
        code = {1: 1, 2: 2, math.inf: -1}.get(degree_p)
        if code is None:
            raise ValueError(f"degree_p must be 1, 2 or math.inf, got {degree_p!r}")
        spec = _Spec(group=group, nu_max=nu_max, degree_max=degree_max, n_max=n_max, l_max=l_max,
                     algorithm=algorithm, alg_n=alg_n, degree_p=code, r_cut=r_cut,
                     build_flags=BUILD_HOST_ONLY if host_only else 0, k_max=k_max)
        self._h = _P()
        _check(lib().ace_graph_build(ctypes.byref(spec), ctypes.byref(self._h)))
        self.spec = dict(group=group, nu_max=nu_max, degree_max=degree_max, n_max=n_max,
                         l_max=l_max, algorithm=algorithm, alg_n=alg_n, r_cut=r_cut, degree_p=degree_p,
                         k_max=k_max)
        self.pos_cols = 4 if k_max > 0 else 3
        self.host_only = host_only
        st = self.stats()
        self.P1 = st["n_onep"]
        self.nK = st["n_k"]
        self.n_nodes = st["n_nodes"]
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.ace_graph_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = _Stats()
        _check(lib().ace_graph_info(self._h, ctypes.byref(s)))
        out = {}
        for name, _ in _Stats._fields_:
            v = getattr(s, name)
            out[name] = list(v) if not isinstance(v, int) else v
        return out

    def export(self):
        """(onep [P1,3], node_tuple [V,nu_max], parents [V,2], k_to_node [|K|])."""
        nu = self.spec["nu_max"]
        onep = np.zeros((self.P1, 3), dtype=np.int32)
        tup = np.zeros((self.n_nodes, nu), dtype=np.int32)
        par = np.zeros((self.n_nodes, 2), dtype=np.int32)
        k2n = np.zeros(self.nK, dtype=np.int64)
        _check(lib().ace_graph_export(self._h, onep.ctypes.data, tup.ctypes.data,
                                      par.ctypes.data, k2n.ctypes.data))
        return onep, tup, par, k2n

    def k_tuples(self) -> np.ndarray:
        out = np.zeros((self.nK, self.spec["nu_max"]), dtype=np.int32)
        _check(lib().ace_graph_export_k(self._h, out.ctypes.data))
        return out

    def onep_feature(self) -> np.ndarray:
        """Feature degree k of every one-particle function (ace_graph_export_feature)."""
        out = np.zeros(self.P1, dtype=np.int32)
        _check(lib().ace_graph_export_feature(self._h, out.ctypes.data))
        return out

    def k_degrees(self) -> np.ndarray:
        """Total degree sum_t (n_t + l_t) of every tuple of K (SO(2): n + |m|, torus: |m|)."""
        onep = self.export()[0]
        if self.spec["group"] == GROUP_TORUS:
            deg1 = np.abs(onep[:, 2])
        else:
            deg1 = onep[:, 0] + onep[:, 1] + self.onep_feature()   # SO(2): the l column holds |m|
        kt = self.k_tuples()
        d = np.where(kt >= 0, deg1[np.maximum(kt, 0)], 0)
        return d.sum(axis=1)

    SCHEDULE_KEYS = ("row_chunk", "tree_chunk", "hot_columns", "bank_schedule", "block_threads",
                     "schedule", "term_chunk", "pair_slots", "env_per_block")

    def get_schedule(self) -> dict:
        """Schedule options (ace_graph_get_schedule); "schedule" is a name of SCHEDULES."""
        o = _Opts()
        _check(lib().ace_graph_get_schedule(self._h, ctypes.byref(o)))
        d = {k: getattr(o, k) for k in self.SCHEDULE_KEYS}
        d["schedule"] = {v: k for k, v in SCHEDULES.items()}[d["schedule"]]
        return d

    def set_schedule(self, **opts):
        """Rebuild the evaluation schedule (ace_graph_set_schedule); unspecified
        options keep their current values."""
        cur = self.get_schedule()
        cur.update(opts)
        if isinstance(cur["schedule"], str):
            cur["schedule"] = SCHEDULES[cur["schedule"]]
        o = _Opts(**{k: int(cur[k]) for k in self.SCHEDULE_KEYS})
        _check(lib().ace_graph_set_schedule(self._h, ctypes.byref(o)))

    def schedule_kind(self) -> str:
        """'forest', 'remat' or 'layered': the kernel ace_eval_grad uses (ace_debug_schedule)."""
        k = ctypes.c_int32()
        _check(lib().ace_debug_schedule(self._h, ctypes.byref(k), None))
        return _KIND[k.value]

    def schedule_info(self) -> dict:
        """Sizes of the schedule in use (ace_debug_schedule)."""
        k = ctypes.c_int32()
        info = np.zeros(16, dtype=np.int64)
        _check(lib().ace_debug_schedule(self._h, ctypes.byref(k), info.ctypes.data))
        if k.value == 2:
            names = ["nslot", "slices", "entry_pos", "entry_real", "items", "fwd_slices", "fwd_entry_pos",
                     "fwd_entry_real", "hot0", "hot1", "hot2", "hot3", "pairs", "bank_cost_x1000",
                     "folded_entry_real", "push_bank_load_x1000"]
        else:
            names = ["nslot", "tree_slices", "child_pos", "child_real", "row_slices", "entry_pos",
                     "entry_real", "grandchildren", "hot0", "hot1", "hot2", "hot3", "full_adjoint",
                     "bank_cost_rows_x1000", "bank_cost_children_x1000", "folded_real"]
        return {"kind": _KIND[k.value], **{n: int(v) for n, v in zip(names, info) if n}}

    def forest_eval_host(self, coeffs: np.ndarray, A: np.ndarray, folded: bool = False):
        """Host emulation of the forest kernel (ace_debug_forest_eval):
        coeffs [|K|] float64, A [E, P1] complex -> (phi [E], Abar [E, P1]);
        folded: the schedule with conjugate pairs folded (exact only for conjugate-symmetric A)."""
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        E = A.shape[0]
        Ar = np.ascontiguousarray(np.stack([A.real, A.imag], -1), dtype=np.float64)
        phi = np.zeros((E, 2))
        ab = np.zeros((E, self.P1, 2))
        _check(lib().ace_debug_forest_eval(self._h, c.ctypes.data, E, Ar.ctypes.data, phi.ctypes.data,
                                           ab.ctypes.data, int(folded)))
        return phi[:, 0] + 1j * phi[:, 1], ab[..., 0] + 1j * ab[..., 1]

    def remat_eval_host(self, coeffs: np.ndarray, A: np.ndarray, folded: bool = False):
        """Host emulation of the remat kernel (ace_debug_remat_eval), as forest_eval_host;
        folded: the schedules with conjugate pairs folded (exact only for conjugate-symmetric A)."""
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        E = A.shape[0]
        Ar = np.ascontiguousarray(np.stack([A.real, A.imag], -1), dtype=np.float64)
        phi = np.zeros((E, 2))
        ab = np.zeros((E, self.P1, 2))
        _check(lib().ace_debug_remat_eval(self._h, c.ctypes.data, E, Ar.ctypes.data, phi.ctypes.data,
                                          ab.ctypes.data, int(folded)))
        return phi[:, 0] + 1j * phi[:, 1], ab[..., 0] + 1j * ab[..., 1]

    def workspace_size(self, n_env: int, n_nbr: int = 0, flags: int = 0) -> int:
        out = _SZ()
        _check(lib().ace_workspace_size(self._h, int(n_env), int(n_nbr), int(flags), ctypes.byref(out)))
        return int(out.value)

    def workspace(self, n_env: int, device, flags: int = 0):
        """A cached device workspace of at least workspace_size(n_env, flags=flags) bytes."""
        import torch
        need = self.workspace_size(n_env, flags=flags)
        key = str(device)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
            self._ws[key] = ws
        return ws


# ---------------------------------------------------------------------------
def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _check_coeffs(g: "Graph", coeffs):
    if coeffs.dim() != 1 or coeffs.numel() != g.nK:
        raise ValueError(f"coeffs must have shape [{g.nK}] (one per tuple of K), got {tuple(coeffs.shape)}")


def _check_batch(offsets, pos, check: bool, cols: int = 3):
    if offsets.dim() != 1 or offsets.numel() < 1:
        raise ValueError("offsets must be a 1-d tensor of n_env + 1 entries")
    if pos.dim() != 2 or pos.shape[1] != cols:
        raise ValueError(f"pos must have shape [n_nbr, {cols}], got {tuple(pos.shape)}")
    if check and offsets.numel() > 1:
        last = int(offsets[-1].item())
        if last != pos.shape[0]:
            raise ValueError(f"offsets[-1] = {last} but pos has {pos.shape[0]} rows")


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_result(ws, device):
    """Wait for the call and read its device-side offsets validation (ACE_FLAG_CHECK)."""
    import torch
    torch.cuda.current_stream(device).synchronize()
    _check(lib().ace_check_offsets_result(ws.data_ptr()))


def basis(g: Graph, offsets, pos):
    """A[e, i] (ace_basis); returns float64 [E, P1, 2]."""
    import torch
    _dev(offsets, torch.int32, "offsets")
    _dev(pos, torch.float64, "pos")
    _check_batch(offsets, pos, True, g.pos_cols)
    E = offsets.numel() - 1
    A = torch.empty((E, g.P1, 2), dtype=torch.float64, device=pos.device)
    _check(lib().ace_basis(g.handle, E, offsets.data_ptr(), pos.data_ptr(), A.data_ptr(),
                           _stream(pos.device)))
    return A


def contract(g: Graph, coeffs, A, *, with_grad: bool = False, naive: bool = False,
             layered: bool = False, conj_symmetric: bool = False):
    """phi [E,2] (and Abar [E,P1,2]) from given one-particle values A [E,P1,2].
    conj_symmetric: A has the symmetry of ace_basis output (ACE_FLAG_CONJ_SYMMETRIC),
    so conjugate pairs may be folded; Abar is then a Re-gradient equivalent."""
    import torch
    _dev(coeffs, torch.float64, "coeffs")
    _dev(A, torch.float64, "A")
    _check_coeffs(g, coeffs)
    if A.dim() != 3 or A.shape[1] != g.P1 or A.shape[2] != 2:
        raise ValueError(f"A must have shape [n_env, {g.P1}, 2], got {tuple(A.shape)}")
    E = A.shape[0]
    phi = torch.empty((E, 2), dtype=torch.float64, device=A.device)
    Abar = torch.empty_like(A) if with_grad else None
    flags = ((FLAG_NAIVE if naive else 0) | (FLAG_LAYERED if layered else 0)
             | (FLAG_CONJ_SYMMETRIC if conj_symmetric else 0))
    ws = g.workspace(E, A.device, flags)
    _check(lib().ace_contract(g.handle, coeffs.data_ptr(), E, A.data_ptr(), phi.data_ptr(),
                              Abar.data_ptr() if Abar is not None else None,
                              ws.data_ptr(), ws.numel(), flags, _stream(A.device)))
    return (phi, Abar) if with_grad else phi


def eval(g: Graph, coeffs, offsets, pos, *, naive: bool = False, check: bool = False, out=None,
         layered: bool = False, unfolded: bool = False):
    """phi [E, 2] = (Re, Im) by ace_eval."""
    import torch
    _dev(coeffs, torch.float64, "coeffs")
    _dev(offsets, torch.int32, "offsets")
    _dev(pos, torch.float64, "pos")
    _check_coeffs(g, coeffs)
    _check_batch(offsets, pos, check, g.pos_cols)
    E = offsets.numel() - 1
    phi = out if out is not None else torch.empty((E, 2), dtype=torch.float64, device=pos.device)
    flags = ((FLAG_NAIVE if naive else 0) | (FLAG_CHECK if check else 0) | (FLAG_LAYERED if layered else 0)
             | (FLAG_UNFOLDED if unfolded else 0))
    ws = g.workspace(E, pos.device, flags)
    _check(lib().ace_eval(g.handle, coeffs.data_ptr(), E, offsets.data_ptr(), pos.data_ptr(),
                          phi.data_ptr(), ws.data_ptr(), ws.numel(), flags, _stream(pos.device)))
    if check and E > 0:
        _check_result(ws, pos.device)
    return phi


def eval_grad(g: Graph, coeffs, offsets, pos, *, naive: bool = False, check: bool = False,
              out=None, layered: bool = False, unfolded: bool = False):
    """(phi [E, 2], grad [N, 3]) by ace_eval_grad; grad = d Re(phi_e)/d r_j."""
    import torch
    _dev(coeffs, torch.float64, "coeffs")
    _dev(offsets, torch.int32, "offsets")
    _dev(pos, torch.float64, "pos")
    _check_coeffs(g, coeffs)
    _check_batch(offsets, pos, check, g.pos_cols)
    E = offsets.numel() - 1
    if out is not None:
        phi, grad = out
    else:
        phi = torch.empty((E, 2), dtype=torch.float64, device=pos.device)
        grad = torch.empty((pos.shape[0], 3), dtype=torch.float64, device=pos.device)
    flags = ((FLAG_NAIVE if naive else 0) | (FLAG_CHECK if check else 0) | (FLAG_LAYERED if layered else 0)
             | (FLAG_UNFOLDED if unfolded else 0))
    ws = g.workspace(E, pos.device, flags)
    _check(lib().ace_eval_grad(g.handle, coeffs.data_ptr(), E, offsets.data_ptr(), pos.data_ptr(),
                               phi.data_ptr(), grad.data_ptr(), ws.data_ptr(), ws.numel(), flags,
                               _stream(pos.device)))
    if check and E > 0:
        _check_result(ws, pos.device)
    return phi, grad


def eval_grad_noalloc(g: Graph, coeffs, offsets, pos, phi, grad, *, naive: bool = False):
    """ace_eval_grad_noalloc into caller-allocated phi [E, 2] and grad [N, 3]:
    the library's fixed device workspace, no allocation in the call."""
    import torch
    _dev(coeffs, torch.float64, "coeffs")
    _dev(offsets, torch.int32, "offsets")
    _dev(pos, torch.float64, "pos")
    _dev(phi, torch.float64, "phi")
    _dev(grad, torch.float64, "grad")
    _check_coeffs(g, coeffs)
    _check_batch(offsets, pos, False, g.pos_cols)
    E = offsets.numel() - 1
    if tuple(phi.shape) != (E, 2) or tuple(grad.shape) != (pos.shape[0], 3):
        raise ValueError("phi must be [n_env, 2] and grad [n_nbr, 3]")
    _check(lib().ace_eval_grad_noalloc(g.handle, coeffs.data_ptr(), E, offsets.data_ptr(), pos.data_ptr(),
                                       phi.data_ptr(), grad.data_ptr(), FLAG_NAIVE if naive else 0,
                                       _stream(pos.device)))
    return phi, grad


def _autograd():
    import torch

    class AceEnergy(torch.autograd.Function):
        """Re(phi_e) per environment; backward scatters grad_out[e] * g_j.

        forward(pos [N,3] f64 (or [N,4] with a feature column), offsets [E+1] i32,
        coeffs [|K|] f64, graph)
        The gradient with respect to the positions comes from ace_eval_grad
        (the feature column gets zero); offsets, coeffs and the graph get
        none.  Double backward is not supported.
        """

        @staticmethod
        def forward(ctx, pos, offsets, coeffs, graph):
            phi, grad = eval_grad(graph, coeffs, offsets, pos.detach().contiguous())
            ctx.save_for_backward(grad, offsets)
            ctx.pos_cols = pos.shape[1]
            return phi[:, 0].clone()

        @staticmethod
        @torch.autograd.function.once_differentiable
        def backward(ctx, grad_out):
            grad, offsets = ctx.saved_tensors
            counts = (offsets[1:] - offsets[:-1]).long()
            w = torch.repeat_interleave(grad_out.contiguous(), counts, output_size=grad.shape[0])
            g = grad * w[:, None]
            if ctx.pos_cols == 4:
                g = torch.cat([g, torch.zeros_like(g[:, :1])], dim=1)
            return g, None, None, None

    return AceEnergy


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _autograd()
        return getattr(_Lazy._cls, name)


AceEnergy = _Lazy()
