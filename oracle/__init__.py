"""Plain FP64 CPU oracle for the recursive sparse-symmetric contraction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.  The
oracle shares no code, table or helper with the GPU path: it re-derives every
quantity from the definitions in the paper (Kaliuzhnyi & Ortner, "Optimal
Evaluation of Symmetry-Adapted n-Correlations Via Recursive Contraction of
Sparse Symmetric Tensors", arXiv:2202.04140) in the most direct form.

Modules
  indexsets    one-particle index lists, invariant tuple sets K_G(nu, D),
               integer partitions (Sec. 2.2-2.5, Sec. 3, Sec. 5.1)
  graph        Algorithm 1 and Algorithm 2 node insertion (Sec. 2.6, 3.2, 3.3)
  onebody      radial basis R_n, complex spherical harmonics Y_l^m, pooled
               A_nlm and their gradients (Sec. 2.1, 2.4)
  contraction  naive phi = sum_k c_k prod_t A_{k_t} and its gradient
               (Eq. (1.1) / Eq. (2.1))

Every function states the passage it follows.  Functions whose result is not
pinned by an independent check say "parity unpinned" in their docstring.
"""
