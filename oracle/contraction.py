"""Naive evaluation of the contraction and of its gradient.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. (1.1) / Eq. (2.1):  phi = sum_{k in K} c_k A_k,  A_k = prod_t A_{k_t}.
Every product is formed directly, left to right, tuple by tuple; no
intermediate product is shared between tuples (that sharing is exactly what
the recursive method adds, so the oracle must not use it).

Derivatives (not in the paper, needed for forces):
  Abar_i = d phi / d A_i = sum_k c_k sum_{t: k_t = i} prod_{s != t} A_{k_s}
  d Re(phi) / d r_j = Re sum_i Abar_i d A_i / d r_j
                    = Re sum_i Abar_i grad phi_i(r_j)      (r_j in env e)
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .onebody import onebody_gradients, pooled_A

CHUNK = 2048


def _group_by_length(tuples):
    """Split K (list of index tuples) into (positions, index array) per length."""
    groups = {}
    for q, k in enumerate(tuples):
        groups.setdefault(len(k), []).append(q)
    out = []
    for nu in sorted(groups):
        qs = np.asarray(groups[nu], dtype=np.int64)
        idx = np.asarray([tuples[q] for q in qs], dtype=np.int64).reshape(len(qs), nu)
        out.append((nu, qs, idx))
    return out


def _neumaier_add(s, comp, x):
    """One step of Neumaier's compensated summation, elementwise."""
    t = s + x
    big = np.abs(s) >= np.abs(x)
    comp = comp + np.where(big, (s - t) + x, (x - t) + s)
    return t, comp


def phi_naive(tuples, coeffs, A: np.ndarray) -> np.ndarray:
    """phi[e] = sum_k c_k prod_t A[e, k_t] for every row e of A ([E, P1] complex).

    Real and imaginary parts are summed separately over chunks with
    compensated summation; inside a chunk the sum is a dot product.
    """
    A = np.asarray(A, dtype=np.complex128)
    coeffs = np.asarray(coeffs, dtype=np.float64)
    E = A.shape[0]
    sr, cr = np.zeros(E), np.zeros(E)
    si, ci = np.zeros(E), np.zeros(E)
    for nu, qs, idx in _group_by_length(tuples):
        for c0 in range(0, len(qs), CHUNK):
            sl = slice(c0, c0 + CHUNK)
            prod = A[:, idx[sl, 0]].copy()
            for t in range(1, nu):
                prod *= A[:, idx[sl, t]]
            part = prod @ coeffs[qs[sl]]
            sr, cr = _neumaier_add(sr, cr, part.real)
            si, ci = _neumaier_add(si, ci, part.imag)
    return (sr + cr) + 1j * (si + ci)


def abar_naive(tuples, coeffs, A: np.ndarray) -> np.ndarray:
    """Abar[e, i] = d phi[e] / d A[e, i] by the product rule, tuple by tuple."""
    A = np.asarray(A, dtype=np.complex128)
    coeffs = np.asarray(coeffs, dtype=np.float64)
    E, P1 = A.shape
    out = np.zeros((E, P1), dtype=np.complex128)
    for nu, qs, idx in _group_by_length(tuples):
        for c0 in range(0, len(qs), CHUNK):
            sl = slice(c0, c0 + CHUNK)
            ii = idx[sl]
            cc = coeffs[qs[sl]]
            for t in range(nu):
                others = np.ones((E, len(ii)), dtype=np.complex128)
                for s in range(nu):
                    if s != t:
                        others *= A[:, ii[:, s]]
                contrib = others * cc[None, :]
                # scatter-add column q of contrib into Abar[:, ii[q, t]]:
                # a product with the one-hot matrix onehot[q, ii[q, t]] = 1
                onehot = sp.csr_matrix((np.ones(len(ii)), (np.arange(len(ii)), ii[:, t])),
                                       shape=(len(ii), P1))
                out += np.asarray((onehot.T @ contrib.T).T)
    return out


def grad_naive(labels, tuples, coeffs, offsets, pos, r_cut: float):
    """phi[e] and g[j] = d Re(phi_e) / d r_j for all neighbours; ([E], [N, 3])."""
    offsets = np.asarray(offsets)
    pos = np.asarray(pos, dtype=np.float64)
    A = pooled_A(labels, offsets, pos, r_cut)
    phi = phi_naive(tuples, coeffs, A)
    Abar = abar_naive(tuples, coeffs, A)
    dphi = onebody_gradients(labels, pos, r_cut)  # [N, P1, 3]
    g = np.zeros((pos.shape[0], 3))
    for e in range(len(offsets) - 1):
        a, b = int(offsets[e]), int(offsets[e + 1])
        if b > a:
            g[a:b] = np.real(np.einsum("i,jid->jd", Abar[e], dphi[a:b]))
    return phi, g


def eval_naive(labels, tuples, coeffs, offsets, pos, r_cut: float) -> np.ndarray:
    """phi[e] for every environment of a CSR batch (Eq. (2.1))."""
    A = pooled_A(labels, offsets, pos, r_cut)
    return phi_naive(tuples, coeffs, A)
