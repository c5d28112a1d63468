// gfx950 kernels of the evaluator.  All arithmetic is binary64 on the
// vector ALU: the DAG is a chain of sparse complex products, not a dense
// contraction, so no matrix-core instruction is used.
//
//   basis_kernel   A_{nlm} = sum_j R_n(|r_j|) Y_l^m(r_j/|r_j|)   (Sec. 2.1, 2.4)
//   dag_kernel     x_v = x_a * x_b over the DAG layers, phi = sum_k c_k x_k,
//                  and optionally the reverse pass giving dphi/dA   (Sec. 2.6)
//   naive_kernel   phi = sum_k c_k prod_t A_{k_t} tuple by tuple     (Eq. (1.1))
//   grad_kernel    d Re(phi)/d r_j = Re sum_i Abar_i grad(R_n Y_l^m)(r_j)
//   planar_basis_kernel, planar_grad_kernel  the same for the torus and SO(2)
//   forest_kernel  the DAG with one-particle and order-2 values resident in
//                  LDS and the higher nodes walked in registers, forward
//                  and reverse in one pass (the main schedule)
//   remat_kernel   the DAG with only one-particle values resident and the
//                  parents of every term recomputed (large DAGs)
#include "ace_kernels.hpp"

namespace ace {

// ---------------------------------------------------------------------------
// complex helpers (double2 = (re, im))
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// acc += a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc += s * a   (s real)
__device__ __forceinline__ double2 rfma(double s, double2 a, double2 acc) {
  acc.x = fma(s, a.x, acc.x);
  acc.y = fma(s, a.y, acc.y);
  return acc;
}

// Sum of one double2 per thread over the block, in a fixed order.
// `scratch` needs blockDim.x / 64 entries.  Result valid in thread 0.
__device__ __forceinline__ double2 block_sum(double2 v, double2* scratch) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) scratch[wid] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) {
      s.x += scratch[w].x;
      s.y += scratch[w].y;
    }
  }
  __syncthreads();
  return s;
}

// Sum of one double2 over the 64 lanes of a wave (every lane gets the sum).
__device__ __forceinline__ double2 wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// ---------------------------------------------------------------------------
// coefficients in schedule order, once per call (the DAG launches read them
// at the positions of their schedules)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prep_range(const PrepArgs& p, int64_t i0, int64_t stride) {
  for (int64_t i = i0; i < p.n; i += stride) {
    const int k = p.kmap[i];
    p.cs[i] = k >= 0 ? p.coeffs[k] : (k == -1 ? 0.0 : 2.0 * p.coeffs[-2 - k]);
  }
}

// Folded coefficients of a conjugate pair {k, kbar} (Re and Im weights):
// (c_k + c_kbar, c_k - c_kbar); a self-conjugate tuple gives (c_k, c_k).
// kmap: k >= 0, -1 (padding: 0), or -2-k (doubled diagonal); kbar < 0: self.
__device__ __forceinline__ void prep_fold_range(const PrepFoldArgs& p, int64_t i0, int64_t stride) {
  for (int64_t i = i0; i < p.n; i += stride) {
    const int k = p.kmap[i], kb = p.kbar[i];
    double2 r = make_double2(0.0, 0.0);
    if (k != -1) {
      const int q = k >= 0 ? k : -2 - k;
      const double sc = k >= 0 ? 1.0 : 2.0;
      const double a = p.coeffs[q];
      const double b = kb >= 0 ? p.coeffs[kb] : a;
      r = kb >= 0 ? make_double2(sc * (a + b), sc * (a - b)) : make_double2(sc * a, sc * a);
    }
    p.cs[i] = r;
  }
}

// the preparation a DAG launch needs, spread over every thread of a grid
__device__ __forceinline__ void prep_on_grid(const CoefPrep& c) {
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (c.mode == CoefPrep::kFold)
    prep_fold_range(c.fold, i0, stride);
  else if (c.mode == CoefPrep::kPlain)
    prep_range(c.plain, i0, stride);
}

// ---------------------------------------------------------------------------
// device-side validation of CSR offsets (ACE_FLAG_CHECK)
// ---------------------------------------------------------------------------
// status = 0 if offsets[0] == 0 and offsets[0..n_env] is non-decreasing,
// 1 if offsets[0] != 0, 2 if a later entry decreases.  One block; always
// writes status, so no clearing is needed.
__global__ __launch_bounds__(1024) void check_offsets_kernel(const int32_t* offsets, int64_t n_env, int32_t* status) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = offsets[0] != 0 ? 1 : 0;
  __syncthreads();
  int mine = 0;
  for (int64_t e = threadIdx.x; e < n_env; e += blockDim.x)
    if (offsets[e + 1] < offsets[e]) mine = 2;
  if (mine) atomicMax(&bad, mine);
  __syncthreads();
  if (threadIdx.x == 0) *status = bad;
}

// Environments a basis or gradient launch reads: none when a validation
// ahead of it on the stream found the offsets invalid.
__device__ __forceinline__ int64_t gated_envs(int64_t n_env, const int32_t* gate) {
  return gate == nullptr || *gate == 0 ? n_env : 0;
}

// ---------------------------------------------------------------------------
// one-particle basis
// ---------------------------------------------------------------------------
constexpr int kBasisBlock = 256;

// One-particle basis.  Per environment, in chunks of neighbours: a table of
// T_n(cos(pi r / r_cut)) and Y_l^m (m >= 0) per neighbour is built in LDS by
// (neighbour, m) lanes, each running the Legendre recurrence in l for its m
// (Y_l^m = q_l^m(z) (x + i y)^m with q_m^m = start_m and
// q_l^m = A_lm z q_{l-1}^m - B_lm q_{l-2}^m; normalisation and
// Condon-Shortley phase are folded into the coefficients on the host; the
// form has no division by sin(theta)).  Then one lane per one-particle
// function i with m_i >= 0 accumulates R_{n_i} Y_{l_i}^{m_i} over the chunk
// and also adds the sums, with the signs of Y_l^{-m} = (-1)^m conj(Y_l^m),
// to its -m partner.
// FEAT: a feature factor T_k(mu) per function (Sec. 5.4); without it the
// radial factor is T_n alone.
template <bool FEAT>
__global__ __launch_bounds__(kBasisBlock) void basis_kernel(BasisArgs p) {
  extern __shared__ double lds_b[];
  const int L = p.l_max;
  const int NY = (L + 1) * (L + 2) / 2;
  const int K1 = FEAT ? p.k_max + 1 : 1;
  // doubles per neighbour: T_n(cos), T_k(mu), Y; odd, so that lanes writing
  // different neighbours' rows spread over the LDS banks
  const int stride = ((p.n_max + 1) + K1 + 2 * NY) | 1;
  const int chunk = blockDim.x / (L + 1);           // neighbours per chunk
  double2* acc = reinterpret_cast<double2*>(lds_b);  // [P1]
  double* tab = lds_b + 2 * p.P1;                    // [chunk][stride]
  const double* cA = p.ycoef;
  const double* cB = p.ycoef + NY;
  const double* cS = p.ycoef + 2 * NY;
  // the coefficient preparation of the DAG launch that follows (independent
  // of this kernel's own work; one launch fewer per step)
  prep_on_grid(p.prep);
  const int64_t n_env = gated_envs(p.n_env, p.gate);
  for (int64_t e = blockIdx.x; e < n_env; e += gridDim.x) {
    const int j0 = p.offsets[e];
    const int J = p.offsets[e + 1] - j0;
    for (int i = threadIdx.x; i < p.P1; i += blockDim.x) acc[i] = make_double2(0.0, 0.0);
    for (int c0 = 0; c0 < J; c0 += chunk) {
      const int nc = min(chunk, J - c0);
      __syncthreads();
      const int jj = threadIdx.x / (L + 1), m = threadIdx.x % (L + 1);
      if (jj < nc) {
        const double* r = p.pos + p.pos_stride * (int64_t)(j0 + c0 + jj);
        const double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        const double inv = 1.0 / rr;
        const double x = r[0] * inv, y = r[1] * inv, z = r[2] * inv;
        double* t = tab + jj * stride;
        if (m == 0) {
          const double c = cos(M_PI * rr / p.r_cut);
          double t0 = 1.0, t1 = c;
          t[0] = 1.0;
          if (p.n_max >= 1) t[1] = c;
          for (int n = 2; n <= p.n_max; ++n) {
            const double t2 = 2.0 * c * t1 - t0;
            t[n] = t2;
            t0 = t1;
            t1 = t2;
          }
          // feature polynomials T_k(mu) (Sec. 5.4)
          double* tk = t + (p.n_max + 1);
          const double mu = K1 > 1 ? r[3] : 0.0;
          double k0 = 1.0, k1 = mu;
          tk[0] = 1.0;
          if (K1 > 1) tk[1] = mu;
          for (int k = 2; k < K1; ++k) {
            const double k2 = 2.0 * mu * k1 - k0;
            tk[k] = k2;
            k0 = k1;
            k1 = k2;
          }
        }
        double pr = 1.0, pi = 0.0;  // (x + i y)^m
        for (int k = 0; k < m; ++k) {
          const double nr = pr * x - pi * y;
          pi = pr * y + pi * x;
          pr = nr;
        }
        double* Y = t + (p.n_max + 1) + K1;
        double q2 = 0.0, q1 = cS[(m * (m + 1)) / 2 + m];
        for (int l = m; l <= L; ++l) {
          const int o = (l * (l + 1)) / 2 + m;
          if (l > m) {
            const double q = cA[o] * z * q1 - cB[o] * q2;
            q2 = q1;
            q1 = q;
          }
          Y[2 * o] = q1 * pr;
          Y[2 * o + 1] = q1 * pi;
        }
      }
      __syncthreads();
      // one lane per function with m >= 0; two neighbours per step into two
      // partial sums (more loads in flight).  The -m partner of an m > 0
      // function gets the same sums with the signs of Y_l^{-m} =
      // (-1)^m conj(Y_l^m) (its own sre, sim) applied.
      for (int q = threadIdx.x; q < p.n_prim; q += blockDim.x) {
        const int i = p.prim[q];
        const OnepInfo o = p.onep[i];
        const int ro = o.n, ko = p.n_max + 1 + o.k, yo = (p.n_max + 1) + K1 + 2 * o.yoff;
        double ax0 = 0.0, ay0 = 0.0, ax1 = 0.0, ay1 = 0.0;
        int k = 0;
        for (; k + 1 < nc; k += 2) {
          const double* t0 = tab + k * stride;
          const double* t1 = t0 + stride;
          const double R0 = FEAT ? t0[ro] * t0[ko] : t0[ro], R1 = FEAT ? t1[ro] * t1[ko] : t1[ro];
          ax0 = fma(R0, t0[yo], ax0);
          ay0 = fma(R0, t0[yo + 1], ay0);
          ax1 = fma(R1, t1[yo], ax1);
          ay1 = fma(R1, t1[yo + 1], ay1);
        }
        if (k < nc) {
          const double* t0 = tab + k * stride;
          const double R0 = FEAT ? t0[ro] * t0[ko] : t0[ro];
          ax0 = fma(R0, t0[yo], ax0);
          ay0 = fma(R0, t0[yo + 1], ay0);
        }
        const double sx = ax0 + ax1, sy = ay0 + ay1;
        double2 a = acc[i];
        a.x = fma((double)o.sre, sx, a.x);
        a.y = fma((double)o.sim, sy, a.y);
        acc[i] = a;
        if (o.neg >= 0) {
          const OnepInfo on = p.onep[o.neg];
          double2 b = acc[o.neg];
          b.x = fma((double)on.sre, sx, b.x);
          b.y = fma((double)on.sim, sy, b.y);
          acc[o.neg] = b;
        }
      }
    }
    __syncthreads();
    double2* Ae = p.A + e * p.P1;
    for (int i = threadIdx.x; i < p.P1; i += blockDim.x) Ae[i] = acc[i];
    __syncthreads();
  }
}

template __global__ void basis_kernel<false>(BasisArgs);
template __global__ void basis_kernel<true>(BasisArgs);

// ---------------------------------------------------------------------------
// DAG forward + reverse pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ void atomic_cadd(double2* addr, double2 v) {
  atomicAdd(&addr->x, v.x);
  atomicAdd(&addr->y, v.y);
}

__device__ __forceinline__ double coef_of(const double* coeffs, int k) {
  return k >= 0 ? coeffs[k] : 0.0;
}

// XL: value arena in LDS; AL: adjoint arena in LDS.  One block per
// environment at a time (grid-stride over environments).
template <bool XL, bool AL>
__global__ __launch_bounds__(256) void dag_kernel(DagArgs p) {
  extern __shared__ double2 lds[];
  const int nl = (XL ? p.slots : 0) + (AL ? p.slots : 0);
  double2* red = lds + nl;
  double2* x = XL ? lds : p.arena_x + (int64_t)blockIdx.x * p.slots;
  double2* ab = AL ? lds + (XL ? p.slots : 0) : p.arena_ab + (int64_t)blockIdx.x * p.slots;
  const int P1 = p.P1;
  for (int64_t e = blockIdx.x; e < p.n_env; e += gridDim.x) {
    const double2* Ae = p.A + e * P1;
    for (int i = threadIdx.x; i < P1; i += blockDim.x) x[i] = Ae[i];
    __syncthreads();
    double2 acc = make_double2(0.0, 0.0);
    for (int i = threadIdx.x; i < P1; i += blockDim.x) {
      const int k = p.leaf_k[i];
      if (k >= 0) acc = rfma(p.coeffs[k], x[i], acc);
    }
    for (int L = 1; L <= p.depth; ++L) {
      for (int i = p.st_off[L] + threadIdx.x; i < p.st_off[L + 1]; i += blockDim.x) {
        const int2 ab2 = p.st_ab[i];
        const double2 v = cmul(x[ab2.x], x[ab2.y]);
        x[P1 + i] = v;
        acc = rfma(coef_of(p.coeffs, p.st_k[i]), v, acc);
      }
      for (int i = p.cl_off[L] + threadIdx.x; i < p.cl_off[L + 1]; i += blockDim.x) {
        const int2 ab2 = p.cl_ab[i];
        const double2 v = cmul(x[ab2.x], x[ab2.y]);
        acc = rfma(p.coeffs[p.cl_k[i]], v, acc);
      }
      __syncthreads();
    }
    const double2 phi = block_sum(acc, red);
    if (threadIdx.x == 0) p.phi[e] = phi;

    if (p.Abar != nullptr) {
      // reverse pass: abar_s = d phi / d x_s, pushed from children to parents
      // layer by layer, top down (every child of a layer-L node lies above L)
      for (int s = threadIdx.x; s < p.slots; s += blockDim.x) {
        const int k = s < P1 ? p.leaf_k[s] : p.st_k[s - P1];
        ab[s] = make_double2(coef_of(p.coeffs, k), 0.0);
      }
      __syncthreads();
      for (int L = p.depth; L >= 1; --L) {
        for (int i = p.cl_off[L] + threadIdx.x; i < p.cl_off[L + 1]; i += blockDim.x) {
          const int2 ab2 = p.cl_ab[i];
          const double c = p.coeffs[p.cl_k[i]];
          const double2 xa = x[ab2.x], xb = x[ab2.y];
          atomic_cadd(&ab[ab2.x], make_double2(c * xb.x, c * xb.y));
          atomic_cadd(&ab[ab2.y], make_double2(c * xa.x, c * xa.y));
        }
        for (int i = p.st_off[L] + threadIdx.x; i < p.st_off[L + 1]; i += blockDim.x) {
          const int2 ab2 = p.st_ab[i];
          const double2 w = ab[P1 + i];
          atomic_cadd(&ab[ab2.x], cmul(w, x[ab2.y]));
          atomic_cadd(&ab[ab2.y], cmul(w, x[ab2.x]));
        }
        __syncthreads();
      }
      double2* Be = p.Abar + e * P1;
      for (int i = threadIdx.x; i < P1; i += blockDim.x) Be[i] = ab[i];
    }
    __syncthreads();
  }
}

template __global__ void dag_kernel<true, true>(DagArgs);
template __global__ void dag_kernel<true, false>(DagArgs);
template __global__ void dag_kernel<false, false>(DagArgs);

// ---------------------------------------------------------------------------
// naive per-tuple evaluation (the baseline): phi = sum_k c_k prod_t A_{k_t},
// gradient by prefix / suffix products.  A sits in LDS with one extra slot
// holding 1 for the padding tuples of the last slice of each length.
// ---------------------------------------------------------------------------
// One slice of the naive evaluation: every tuple's product formed from its
// one-particle factors (Eq. (1.1)), nothing shared between tuples.  The
// adjoint of factor t is c_k prod_{s != t} A_{k_s} by prefix and suffix
// products; consecutive tuples of a lane share leading factors (K order), so
// the adjoints of factors 0..NU-2 are summed in registers while the factor
// stays the same and added to LDS when it changes; the last factor's goes to
// LDS at once.
template <int NU, bool GRAD>
__device__ __forceinline__ void naive_slice(const NaiveArgs& p, const double2* x, double2* ab, const int4& sl,
                                            int lane, double2& acc) {
  const int16_t* ip = p.idx + sl.x + lane;
  const double* cp = p.cs + sl.y + lane;
  const int steps = sl.w;
  constexpr int NR = NU > 1 ? NU - 1 : 1;
  int rs[NR];
  double2 rv[NR];
#pragma unroll
  for (int t = 0; t < NR; ++t) {
    rs[t] = -1;
    rv[t] = make_double2(0.0, 0.0);
  }
  for (int j = 0; j < steps; ++j) {
    int f[NU];
    double2 v[NU];
#pragma unroll
    for (int t = 0; t < NU; ++t) f[t] = ip[(j * NU + t) * 64];
    const double c = cp[j * 64];
#pragma unroll
    for (int t = 0; t < NU; ++t) v[t] = x[f[t]];
    double2 pre[NU];   // pre[t] = prod_{s < t} v[s]
    pre[0] = make_double2(1.0, 0.0);
#pragma unroll
    for (int t = 1; t < NU; ++t) pre[t] = t == 1 ? v[0] : cmul(pre[t - 1], v[t - 1]);
    const double2 prod = NU == 1 ? v[0] : cmul(pre[NU - 1], v[NU - 1]);
    acc = rfma(c, prod, acc);
    if (GRAD) {
      double2 suf = make_double2(c, 0.0);
#pragma unroll
      for (int t = NU - 1; t >= 0; --t) {
        const double2 d = t == 0 ? suf : cmul(pre[t], suf);
        if (t == NU - 1) {
          atomic_cadd(&ab[f[t]], d);
        } else {
          if (f[t] != rs[t]) {
            if (rs[t] >= 0) atomic_cadd(&ab[rs[t]], rv[t]);
            rs[t] = f[t];
            rv[t] = d;
          } else {
            rv[t].x += d.x;
            rv[t].y += d.y;
          }
        }
        if (t > 0) suf = cmul(suf, v[t]);
      }
    }
  }
  if (GRAD) {
#pragma unroll
    for (int t = 0; t < NU - 1; ++t)
      if (rs[t] >= 0) atomic_cadd(&ab[rs[t]], rv[t]);
  }
}

constexpr int kNaiveBlock = 256;

template <bool GRAD>
__global__ __launch_bounds__(kNaiveBlock) void naive_kernel(NaiveArgs p) {
  extern __shared__ double2 lds[];
  const int P1 = p.P1;
  double2* x = lds;                // [P1 + 1]
  double2* ab = lds + (P1 + 1);    // [P1 + 1]
  double2* red = ab + (P1 + 1);
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  for (int64_t e = blockIdx.x; e < p.n_env; e += gridDim.x) {
    const double2* Ae = p.A + e * P1;
    for (int i = threadIdx.x; i <= P1; i += blockDim.x) {
      x[i] = i < P1 ? Ae[i] : make_double2(1.0, 0.0);
      if (GRAD) ab[i] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    double2 acc = make_double2(0.0, 0.0);
    for (int s = wid; s < p.n_slices; s += nw) {
      const int4 sl = p.slice[s];
      switch (sl.z) {
        case 1: naive_slice<1, GRAD>(p, x, ab, sl, lane, acc); break;
        case 2: naive_slice<2, GRAD>(p, x, ab, sl, lane, acc); break;
        case 3: naive_slice<3, GRAD>(p, x, ab, sl, lane, acc); break;
        case 4: naive_slice<4, GRAD>(p, x, ab, sl, lane, acc); break;
        case 5: naive_slice<5, GRAD>(p, x, ab, sl, lane, acc); break;
        case 6: naive_slice<6, GRAD>(p, x, ab, sl, lane, acc); break;
        case 7: naive_slice<7, GRAD>(p, x, ab, sl, lane, acc); break;
        default: naive_slice<8, GRAD>(p, x, ab, sl, lane, acc); break;
      }
    }
    const double2 phi = block_sum(acc, red);   // synchronises the block
    if (threadIdx.x == 0) p.phi[e] = phi;
    if (GRAD) {
      double2* Be = p.Abar + e * P1;
      for (int i = threadIdx.x; i < P1; i += blockDim.x) Be[i] = ab[i];
    }
    __syncthreads();
  }
}

template __global__ void naive_kernel<false>(NaiveArgs);
template __global__ void naive_kernel<true>(NaiveArgs);

// ---------------------------------------------------------------------------
// dA/dr chain.
//   grad(R_n Y_l^m)(r) = R_n'(r) u Y_l^m(u) + R_n(r) grad Y_l^m(r)
// With S_l^m(r) = (x + i y)^m Q_l^m(z, rho), rho = |r|^2, a homogeneous
// polynomial of degree l equal to r^l Y_l^m(u) (u = r / |r|),
//   grad Y_l^m(r) = (grad S(u) - l S(u) u) / |r|,
// where Q follows the same recurrence as q with the constant term scaled
// by rho, differentiated in z and rho alongside (no pole singularity).
//
// One wave (one block) per environment.  Its adjoint is staged in LDS per
// (l, m >= 0) with the +m and -m functions already combined into the two
// real weights the gradient needs (see below), in (l, m, n, k) order with
// zeros for absent functions, so the inner loop over n reads one affine
// address; the block of one (l, m) has an odd length nb.
//
// Work is balanced over the lanes: the neighbours are taken in chunks of
// kGradChunk; the (neighbour, m >= 0, l) units of a chunk, neighbour-major
// and m-major, are cut into 64 contiguous ranges, one per lane.  A lane
// walks its range with the Legendre recurrence in l (restarted on a new m,
// warmed up when its range starts inside an m line) and adds its partial
// gradient of each neighbour to an LDS accumulator when it leaves that
// neighbour.  Per-neighbour quantities, T_n and T_n' among them, are
// computed once per chunk into LDS.
// FEAT: a feature factor T_k(mu) per function (Sec. 5.4).
// ---------------------------------------------------------------------------
constexpr int kGradChunk = 16;   // neighbours per chunk
// doubles per neighbour: x, y, z, 1/r, cos, dcos/dr, mu, pad, then (T_n, T_n') for n = 0..n_max
__host__ __device__ constexpr int grad_nbr_doubles(int n_max) { return 8 + 2 * (n_max + 1); }

template <bool FEAT>
__global__ __launch_bounds__(64, 4) void grad_kernel(GradArgs p) {
  extern __shared__ double2 lds[];
  const int L = p.l_max, N = p.n_max;
  const int K1 = FEAT ? p.k_max + 1 : 1;
  const int NY = (L + 1) * (L + 2) / 2;        // (l, m >= 0) units per neighbour
  const int NB = p.nb;                         // entries per (l, m)
  const int ND = NY * NB;
  const int lane = threadIdx.x;
  double2* Ab = lds;                                           // [ND]
  const int NR = grad_nbr_doubles(N);
  double* yc = reinterpret_cast<double*>(lds + ND);            // [3 * NY]
  double* nbr = yc + ((3 * NY + 1) & ~1);                      // [kGradChunk][NR], 16-byte aligned
  double* gacc = nbr + kGradChunk * NR;                        // [kGradChunk][3]
  for (int i = lane; i < 3 * NY; i += 64) yc[i] = p.ycoef[i];
  const double* cA = yc;
  const double* cB = yc + NY;
  const double* cS = yc + 2 * NY;
  const int64_t n_env = gated_envs(p.n_env, p.gate);
  for (int64_t e = blockIdx.x; e < n_env; e += gridDim.x) {
    const int j0 = p.offsets[e];
    const int J = p.offsets[e + 1] - j0;
    if (J <= 0) continue;   // block-uniform
    __syncthreads();
    const double2* Be = p.Abar + e * p.P1;
    // The +m and -m terms of one (n, l, m, k) (Y_l^{-m} = (-1)^m conj(Y_l^m),
    // likewise its gradient; m = 0 counted once) sum to Br Re(g) + Bi Im(g)
    // for g = Y or grad Y with Br = abar.re(+m) + s abar.re(-m),
    // Bi = s abar.im(-m) - abar.im(+m), s = (-1)^m: the staged entry is
    // (Br, Bi).  Four entries per lane at a time: the table loads, then the
    // Abar loads, are all in flight together.
    for (int d0 = lane; d0 < ND; d0 += 4 * 64) {
      int2 src[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) src[r] = d0 + 64 * r < ND ? p.gsrc[d0 + 64 * r] : make_int2(-1, -1);
      double2 vp[4], vm[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int im = src[r].y >= 0 ? src[r].y : -2 - src[r].y;
        vp[r] = src[r].x >= 0 ? Be[src[r].x] : make_double2(0.0, 0.0);
        vm[r] = src[r].y != -1 ? Be[im] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (d0 + 64 * r < ND) {
          const double sg = src[r].y >= 0 ? 1.0 : -1.0;   // vm is 0 where there is no -m
          Ab[d0 + 64 * r] = make_double2(fma(sg, vm[r].x, vp[r].x), fma(sg, vm[r].y, -vp[r].y));
        }
    }
    for (int c0 = 0; c0 < J; c0 += kGradChunk) {
      const int nc = min(kGradChunk, J - c0);
      __syncthreads();
      if (lane < nc) {
        const double* rp = p.pos + p.pos_stride * (int64_t)(j0 + c0 + lane);
        const double rx = rp[0], ry = rp[1], rz = rp[2];
        const double rr = sqrt(rx * rx + ry * ry + rz * rz);
        const double inv = 1.0 / rr;
        const double arg = M_PI * rr / p.r_cut;
        double* nd = nbr + lane * NR;
        const double c = cos(arg);
        nd[0] = rx * inv;
        nd[1] = ry * inv;
        nd[2] = rz * inv;
        nd[3] = inv;
        nd[4] = c;
        nd[5] = -(M_PI / p.r_cut) * sin(arg);
        nd[6] = FEAT ? rp[3] : 0.0;   // invariant feature (Sec. 5.4)
        nd[7] = 0.0;
        // T_n(c) and T_n'(c) by the Chebyshev recurrence
        double* tt = nd + 8;
        double t0 = 1.0, t1 = c, d0 = 0.0, d1 = 1.0;
        tt[0] = 1.0;
        tt[1] = 0.0;
        if (N >= 1) {
          tt[2] = c;
          tt[3] = 1.0;
        }
        for (int n = 2; n <= N; ++n) {
          const double T = 2.0 * c * t1 - t0;
          const double dT = 2.0 * t1 + 2.0 * c * d1 - d0;
          t0 = t1;
          t1 = T;
          d0 = d1;
          d1 = dT;
          tt[2 * n] = T;
          tt[2 * n + 1] = dT;
        }
        gacc[3 * lane] = gacc[3 * lane + 1] = gacc[3 * lane + 2] = 0.0;
      }
      __syncthreads();
      const int U = nc * NY;
      const int u0 = (lane * U) >> 6, u1 = ((lane + 1) * U) >> 6;
      if (u0 < u1) {
        // first unit: neighbour jj, line m, degree l
        int jj = u0 / NY, r = u0 - jj * NY, m = 0;
        while (r >= L + 1 - m) {
          r -= L + 1 - m;
          ++m;
        }
        int l = m + r;
        double x, y, z, inv, dcdr, mu;
        const double* nd = nbr;
        auto load_nbr = [&](int q) {
          nd = nbr + q * NR;
          x = nd[0];
          y = nd[1];
          z = nd[2];
          inv = nd[3];
          dcdr = nd[5];
          mu = nd[6];
        };
        load_nbr(jj);
        // p = (x + i y)^m, q = (x + i y)^(m-1) (0 for m = 0)
        double pr = 1.0, pi = 0.0, qr = 0.0, qi = 0.0;
        for (int k = 0; k < m; ++k) {
          qr = pr;
          qi = pi;
          const double nr = pr * x - pi * y;
          pi = pr * y + pi * x;
          pr = nr;
        }
        // Q, Qz, Qp at l and at l - 1 (Qm, Qzm, Qpm), from l = m
        double Q = cS[(m * (m + 1)) / 2 + m], Qz = 0.0, Qp = 0.0, Qm = 0.0, Qzm = 0.0, Qpm = 0.0;
        auto step_l = [&](int lnew) {
          const int o = (lnew * (lnew + 1)) / 2 + m;
          const double a = cA[o], b = cB[o];
          const double Qn = a * z * Q - b * Qm;
          const double Qzn = a * (Q + z * Qz) - b * Qzm;
          const double Qpn = a * z * Qp - b * (Qm + Qpm);
          Qm = Q;
          Qzm = Qz;
          Qpm = Qp;
          Q = Qn;
          Qz = Qzn;
          Qp = Qpn;
        };
        for (int ll = m + 1; ll <= l; ++ll) step_l(ll);
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int u = u0; u < u1; ++u) {
          // (Br, Bi) = sum_{n,k} (staged entry) T_n T_k, (B1r, B1i) the same with T_n'
          const double2* bc = Ab + ((l * (l + 1)) / 2 + m) * NB;
          double Br = 0.0, Bi = 0.0, B1r = 0.0, B1i = 0.0;
          const double2* tt = reinterpret_cast<const double2*>(nd + 8);   // (T_n, T_n')
#pragma unroll 2
          for (int n = 0; n <= N; ++n) {
            const double2 td = tt[n];
            const double T = td.x, dT = td.y;
            double k0 = 1.0, k1 = mu;
            for (int k = 0; k < K1; ++k) {
              double Tk = 1.0;
              if (FEAT) {
                if (k == 1) {
                  Tk = mu;
                } else if (k >= 2) {
                  Tk = 2.0 * mu * k1 - k0;
                  k0 = k1;
                  k1 = Tk;
                }
              }
              const double w = T * Tk, dw = dT * Tk;
              const double2 cc = bc[n * K1 + k];
              Br = fma(cc.x, w, Br);
              Bi = fma(cc.y, w, Bi);
              B1r = fma(cc.x, dw, B1r);
              B1i = fma(cc.y, dw, B1i);
            }
          }
          // With S = p Q, p = (x + i y)^m, q = (x + i y)^(m-1) at the unit
          // vector u:
          //   grad S = 2 Qp p u + m Q q (1, i, 0) + Qz p e_z,
          //   grad Y = (grad S - l S u) / |r|,  d/dr of the radial part: T_n' dcos/dr,
          // so everything pairs (Br, Bi) with p (P) or q.
          const double P = fma(Br, pr, Bi * pi);
          const double P1 = fma(B1r, pr, B1i * pi);
          const double cu = fma(dcdr * Q, P1, inv * P * (2.0 * Qp - (double)l * Q));
          const double mq = inv * (double)m * Q;
          gx = fma(x, cu, fma(mq, fma(Br, qr, Bi * qi), gx));
          gy = fma(y, cu, fma(mq, fma(Bi, qr, -(Br * qi)), gy));
          gz = fma(z, cu, fma(inv * Qz, P, gz));
          // next unit
          if (l < L) {
            ++l;
            step_l(l);
          } else if (m < L) {
            ++m;
            l = m;
            qr = pr;
            qi = pi;
            const double nr = pr * x - pi * y;
            pi = pr * y + pi * x;
            pr = nr;
            Q = cS[(m * (m + 1)) / 2 + m];
            Qz = Qp = Qm = Qzm = Qpm = 0.0;
          } else {
            atomicAdd(&gacc[3 * jj], gx);
            atomicAdd(&gacc[3 * jj + 1], gy);
            atomicAdd(&gacc[3 * jj + 2], gz);
            gx = gy = gz = 0.0;
            ++jj;
            m = 0;
            l = 0;
            if (jj < nc) load_nbr(jj);
            pr = 1.0;
            pi = qr = qi = 0.0;
            Q = cS[0];
            Qz = Qp = Qm = Qzm = Qpm = 0.0;
          }
        }
        if (jj < nc) {
          atomicAdd(&gacc[3 * jj], gx);
          atomicAdd(&gacc[3 * jj + 1], gy);
          atomicAdd(&gacc[3 * jj + 2], gz);
        }
      }
      __syncthreads();
      if (lane < nc) {
        double* gout = p.grad + 3 * (int64_t)(j0 + c0 + lane);
        gout[0] = gacc[3 * lane];
        gout[1] = gacc[3 * lane + 1];
        gout[2] = gacc[3 * lane + 2];
      }
    }
  }
}

template __global__ void grad_kernel<false>(GradArgs);
template __global__ void grad_kernel<true>(GradArgs);

// ---------------------------------------------------------------------------
// Planar groups (Sec. 2.2 SO(2), Sec. 2.3 torus).  Positions are read as
// (x, y); theta = atan2(y, x) enters only through u = (x + i y)/r.
//   planar_basis_kernel  A_i = sum_j R_{n_i}(r_j) e^{i s m_i theta_j}: per
//                        chunk of neighbours a table of T_n(cos(pi r / r_cut))
//                        and u^{|m|} (repeated products) in LDS, one lane per
//                        neighbour; then one lane per one-particle function
//   planar_grad_kernel   g_j = Re sum_i Abar_i grad phi_i(r_j): per chunk a
//                        table of R_n, R_n', u^{|m|} and grad theta per
//                        neighbour, then the (neighbour, n, |m|) units cut
//                        into contiguous ranges over the block's threads,
//                        partial gradients added to LDS accumulators
//     grad phi = R_n'(r) e r_hat + R_n(r) (i s m) e grad theta,
//     grad theta = (-y, x) / r^2.
// A_{n,-m} is computed with the same operations as A_{n,m} and the opposite
// sign of the imaginary part, so it is exactly conj(A_{n,m}).
// ---------------------------------------------------------------------------
constexpr int kPlanarChunk = 64;   // neighbours per table

__global__ __launch_bounds__(256) void planar_basis_kernel(BasisArgs p) {
  extern __shared__ double lds_p[];
  const bool radial = p.group == 2;
  const int N = p.n_max, M = p.l_max;
  const int stride = ((N + 1) + 2 * (M + 1)) | 1;   // per neighbour: T_n, then (Re, Im) u^m
  const double kr = M_PI / p.r_cut;
  double2* acc = reinterpret_cast<double2*>(lds_p);   // [P1]
  double* tab = lds_p + 2 * p.P1;                      // [kPlanarChunk][stride]
  const int64_t n_env = gated_envs(p.n_env, p.gate);
  for (int64_t e = blockIdx.x; e < n_env; e += gridDim.x) {
    const int j0 = p.offsets[e];
    const int J = p.offsets[e + 1] - j0;
    __syncthreads();
    for (int i = threadIdx.x; i < p.P1; i += blockDim.x) acc[i] = make_double2(0.0, 0.0);
    for (int c0 = 0; c0 < J; c0 += kPlanarChunk) {
      const int nc = min(kPlanarChunk, J - c0);
      __syncthreads();
      if ((int)threadIdx.x < nc) {
        const int64_t j = j0 + c0 + threadIdx.x;
        const double x = p.pos[3 * j], y = p.pos[3 * j + 1];
        const double r = sqrt(x * x + y * y);
        const double c = x / r, sn = y / r;
        double* t = tab + threadIdx.x * stride;
        t[0] = 1.0;
        if (radial && N >= 1) {
          const double X = cos(kr * r);
          double t0 = 1.0, t1 = X;
          t[1] = X;
          for (int n = 2; n <= N; ++n) {
            const double t2 = 2.0 * X * t1 - t0;
            t0 = t1;
            t1 = t2;
            t[n] = t2;
          }
        }
        double er = 1.0, ei = 0.0;
        double* E = t + (N + 1);
        E[0] = 1.0;
        E[1] = 0.0;
        for (int m = 1; m <= M; ++m) {
          const double t2 = er * c - ei * sn;
          ei = er * sn + ei * c;
          er = t2;
          E[2 * m] = er;
          E[2 * m + 1] = ei;
        }
      }
      __syncthreads();
      for (int i = threadIdx.x; i < p.P1; i += blockDim.x) {
        const OnepInfo o = p.onep[i];
        const int ro = radial ? o.n : 0, eo = (N + 1) + 2 * o.am;
        double ar = 0.0, ai = 0.0;
        for (int k = 0; k < nc; ++k) {
          const double* t = tab + k * stride;
          const double R = t[ro];
          ar = fma(R, t[eo], ar);
          ai = fma(R, (double)o.sim * t[eo + 1], ai);
        }
        double2 a = acc[i];
        a.x += ar;
        a.y += ai;
        acc[i] = a;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < p.P1; i += blockDim.x) p.A[e * p.P1 + i] = acc[i];
  }
}

constexpr int kPlanarNbr = 4;   // doubles per neighbour before the R_n table: cos, sin, grad theta

__global__ __launch_bounds__(256) void planar_grad_kernel(GradArgs p) {
  extern __shared__ double2 lds[];
  const bool radial = p.group == 2;
  const double s_exp = radial ? -1.0 : 1.0;
  const int N = radial ? p.n_max : 0, M = p.l_max, W = 2 * M + 1;
  const int stride = (kPlanarNbr + 2 * (N + 1) + 2 * (M + 1)) | 1;   // cos, sin, grad theta, R, R', u^m
  const double kr = M_PI / p.r_cut;
  double2* Ab = lds;                                               // [P1]
  double* tab = reinterpret_cast<double*>(Ab + p.P1);              // [kPlanarChunk][stride]
  double* gacc = tab + kPlanarChunk * stride;                      // [kPlanarChunk][2]
  const int NU = (N + 1) * (M + 1);                                // (n, |m|) units per neighbour
  const int64_t n_env = gated_envs(p.n_env, p.gate);
  for (int64_t e = blockIdx.x; e < n_env; e += gridDim.x) {
    const int j0 = p.offsets[e];
    const int J = p.offsets[e + 1] - j0;
    __syncthreads();
    for (int i = threadIdx.x; i < p.P1; i += blockDim.x) Ab[i] = p.Abar[e * p.P1 + i];
    for (int c0 = 0; c0 < J; c0 += kPlanarChunk) {
      const int nc = min(kPlanarChunk, J - c0);
      __syncthreads();
      if ((int)threadIdx.x < nc) {
        const int64_t j = j0 + c0 + threadIdx.x;
        const double x = p.pos[3 * j], y = p.pos[3 * j + 1];
        const double r2 = x * x + y * y, r = sqrt(r2);
        double* t = tab + threadIdx.x * stride;
        t[0] = x / r;
        t[1] = y / r;
        t[2] = -y / r2;   // grad theta
        t[3] = x / r2;
        double* R = t + kPlanarNbr;          // R_n
        double* dR = R + (N + 1);            // R_n' = n U_{n-1}(X) dX/dr
        R[0] = 1.0;
        dR[0] = 0.0;
        if (radial && N >= 1) {
          const double X = cos(kr * r), dX = -kr * sin(kr * r);
          double tm1 = 1.0, tc = X, um2 = 0.0, um1 = 1.0;   // T_{n-1}, T_n, U_{n-2}, U_{n-1}
          R[1] = X;
          dR[1] = dX;
          for (int n = 2; n <= N; ++n) {
            const double t2 = 2.0 * X * tc - tm1;
            tm1 = tc;
            tc = t2;
            const double u2 = n == 2 ? 2.0 * X : 2.0 * X * um1 - um2;
            um2 = um1;
            um1 = u2;
            R[n] = tc;
            dR[n] = (double)n * um1 * dX;
          }
        }
        double* E = dR + (N + 1);
        const double c = t[0], sn = t[1];
        double er = 1.0, ei = 0.0;
        E[0] = 1.0;
        E[1] = 0.0;
        for (int m = 1; m <= M; ++m) {
          const double t2 = er * c - ei * sn;
          ei = er * sn + ei * c;
          er = t2;
          E[2 * m] = er;
          E[2 * m + 1] = ei;
        }
        gacc[2 * threadIdx.x] = gacc[2 * threadIdx.x + 1] = 0.0;
      }
      __syncthreads();
      const int U = nc * NU;
      const int u0 = (int)(((int64_t)threadIdx.x * U) / blockDim.x);
      const int u1 = (int)(((int64_t)(threadIdx.x + 1) * U) / blockDim.x);
      int jj = -1;
      double gx = 0.0, gy = 0.0;
      for (int u = u0; u < u1; ++u) {
        const int q = u / NU, r = u - q * NU, n = r / (M + 1), m = r - n * (M + 1);
        if (q != jj) {
          if (jj >= 0) {
            atomicAdd(&gacc[2 * jj], gx);
            atomicAdd(&gacc[2 * jj + 1], gy);
          }
          jj = q;
          gx = gy = 0.0;
        }
        const double* t = tab + q * stride;
        const double c = t[0], sn = t[1], gtx = t[2], gty = t[3];
        const double Rn = radial ? t[kPlanarNbr + n] : 1.0;
        const double dRn = radial ? t[kPlanarNbr + (N + 1) + n] : 0.0;
        const double* E = t + kPlanarNbr + 2 * (N + 1);
        const double er = E[2 * m], ei = E[2 * m + 1];
        for (int sg = 1; sg >= (m == 0 ? 1 : -1); sg -= 2) {
          const int i = p.pidx[n * W + M + sg * m];
          if (i < 0) continue;
          // phi = R (er, s * sg * ei) = R E with E = e^{i s (sg m) theta}
          const double qr = er, qi = s_exp * (double)sg * ei;
          const double2 a = Ab[i];
          const double re = a.x * qr - a.y * qi;         // Re(abar E)
          const double im = a.x * qi + a.y * qr;         // Im(abar E)
          // Re(abar * (i s sg m) R E) = -(s sg m) R Im(abar E)
          const double ang = -(s_exp * (double)(sg * m)) * Rn * im;
          gx += dRn * re * c + ang * gtx;
          gy += dRn * re * sn + ang * gty;
        }
      }
      if (jj >= 0) {
        atomicAdd(&gacc[2 * jj], gx);
        atomicAdd(&gacc[2 * jj + 1], gy);
      }
      __syncthreads();
      if ((int)threadIdx.x < nc) {
        const int64_t j = j0 + c0 + threadIdx.x;
        p.grad[3 * j] = gacc[2 * threadIdx.x];
        p.grad[3 * j + 1] = gacc[2 * threadIdx.x + 1];
        p.grad[3 * j + 2] = 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Coefficients in schedule order, once per call.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void prep_kernel(PrepArgs p) {
  prep_range(p, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// ---------------------------------------------------------------------------
// Forest kernel: the DAG evaluated with the one-particle and order-2 node
// values resident in LDS and every higher node computed in registers.
//
// Every product node above order 2 has exactly one parent outside the
// resident set, so those nodes form trees hanging off "roots" (products of
// two resident nodes).  One lane walks one tree (or a chunk of its
// children): x_v = x_a x_b, then each child w = v * s, and for a child with
// children of its own each grandchild g = w * s'.  Childless products of two
// resident nodes form a symmetric sparse matrix M over the resident slots;
// each lane gathers one row chunk y = M x, which gives both the forward
// contribution (phi += x.y / 2) and the adjoint (abar += y) with no atomics.
//
// Where LDS has room (FULL), every resident slot has an adjoint accumulator
// and the order-2 adjoints reach the one-particle ones by one gather per
// one-particle node at the end.  Otherwise order-2 adjoints are not stored:
// a contribution d to abar_u, u = a * b, is forwarded at once to the
// one-particle adjoints (abar_a += d x_b, abar_b += d x_a).  Adjoints are LDS
// accumulators updated with atomics, so the reverse pass is not bitwise
// deterministic (the forward pass is).
// ---------------------------------------------------------------------------
// Adjoint accumulators of one environment in LDS, in two planes of doubles:
// Re abar_s at re[s], Im abar_s at re[n + s].  The LDS serves 8-byte
// atomics a quarter-wave at a time over 16 bank pairs; in a plane the atomic
// on slot s lands on pair s mod 16 (up to a shift), so a quarter whose slots
// are distinct mod 16 is served without conflicts, where with interleaved
// complex values the real parts of 16 slots would share 8 pairs.
struct AdjPlanes {
  double* re;
  int n;
  __device__ __forceinline__ void add(int s, double2 d) const {
    atomicAdd(re + s, d.x);
    atomicAdd(re + n + s, d.y);
  }
  __device__ __forceinline__ double2 get(int s) const { return make_double2(re[s], re[n + s]); }
  __device__ __forceinline__ void set(int s, double2 v) const {
    re[s] = v.x;
    re[n + s] = v.y;
  }
};

__device__ __forceinline__ void push_adj(int P1, const uint32_t* n2, const double2* x, const AdjPlanes& ab, int slot,
                                         double2 d) {
  if (slot <= P1) {
    ab.add(slot, d);
  } else {
    const uint32_t q = n2[slot - P1 - 1];
    const int a = (int)(q & 0xffffu), b = (int)(q >> 16);
    ab.add(a, cmul(d, x[b]));
    ab.add(b, cmul(d, x[a]));
  }
}

// Push with an adjoint accumulator for every resident slot (full mode) or
// forwarding order-2 contributions to the one-particle adjoints at once.
template <bool FULL>
__device__ __forceinline__ void push_r(int P1, const uint32_t* n2, const double2* x, const AdjPlanes& ab, int slot,
                                       double2 d) {
  if (FULL)
    ab.add(slot, d);
  else
    push_adj(P1, n2, x, ab, slot, d);
}

// A coefficient of the forest or remat schedules: c (plain), or (c', c'')
// for a folded conjugate pair (Re and Im weights).
template <bool FOLD>
struct RCoef;
template <>
struct RCoef<false> {
  double c;
};
template <>
struct RCoef<true> {
  double2 c;
};

template <bool FOLD>
__device__ __forceinline__ RCoef<FOLD> load_coef(const double* cs, unsigned i) {
  RCoef<FOLD> r;
  if constexpr (FOLD)
    r.c = reinterpret_cast<const double2*>(cs)[i];
  else
    r.c = cs[i];
  return r;
}

// y1 += c' x (and y2 += c'' x when folded)
template <bool FOLD>
__device__ __forceinline__ void coef_fma(const RCoef<FOLD>& k, double2 v, double2& y1, double2& y2) {
  if constexpr (FOLD) {
    y1 = rfma(k.c.x, v, y1);
    y2 = rfma(k.c.y, v, y2);
  } else {
    y1 = rfma(k.c, v, y1);
  }
}

// The Re weight (the one the adjoint takes).
template <bool FOLD>
__device__ __forceinline__ double re_w(const RCoef<FOLD>& k) {
  if constexpr (FOLD)
    return k.c.x;
  else
    return k.c;
}

// Schedule metadata and coefficients of the forest and remat kernels are
// read with buffer loads: a per-lane byte offset fixed for the whole slice
// and a wave-uniform offset (scalar register) that advances with the entry
// column, so no per-entry address arithmetic runs on the vector ALU.
// Resource word 3 as for raw buffers on CDNA; out-of-range loads return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}
struct EntryBufs {
  __amdgpu_buffer_rsrc_t lo, hi, cs;
};
__device__ __forceinline__ int buf_u16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return (int)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
}
__device__ __forceinline__ uint64_t buf_u64(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// coefficient of entry column index u (wave-uniform part of the coefficient index)
template <bool FOLD>
__device__ __forceinline__ RCoef<FOLD> buf_coef(__amdgpu_buffer_rsrc_t r, int lane, int u) {
  RCoef<FOLD> k;
  if constexpr (FOLD)
    k.c = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16, u * 16, 0));
  else
    k.c = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, lane * 8, u * 8, 0));
  return k;
}

constexpr int kForestBlock = 512;

// FOLD: the folded schedule (one tuple of each conjugate pair, with
// (Re, Im) weights).  Every sum sum_j c_j x_j of the unfolded kernel is then
// kept twice, with the Re weights (t, y, aw: Re phi and the adjoint) and
// with the Im weights (ti, yi, awi: Im phi only), since
// c' Re(u w) + i c'' Im(u w) = Re(u sum c' w) + i Im(u sum c'' w).
// NE environments per block share every schedule and coefficient load
// (each has its own values and adjoints in LDS); a missing last
// environment computes on zeros and writes nothing.
template <bool GRAD, bool GC, bool FULL, bool FOLD, int NE>
__global__ __launch_bounds__(kForestBlock, NE == 1 ? 4 : 2) void forest_kernel(ForestArgs p) {
  extern __shared__ double2 lds[];
  // per environment: values of the resident slots, then adjoints of all
  // resident slots (FULL) or of the one-particle slots only (!FULL); then the
  // order-2 parent table (!FULL) and the reduction scratch
  constexpr bool TAB = GRAD && !FULL;
  const int nab = GRAD ? (FULL ? p.nslot : p.P1 + 1) : 0;
  const int per_env = p.nslot + nab;
  double2* x[NE];
  AdjPlanes ab[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    x[q] = lds + q * per_env;
    ab[q] = AdjPlanes{reinterpret_cast<double*>(x[q] + p.nslot), nab};
  }
  uint32_t* n2 = reinterpret_cast<uint32_t*>(lds + NE * per_env);
  double2* red = reinterpret_cast<double2*>(n2) + (TAB ? (p.N2 + 3) / 4 : 0);
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int P1 = p.P1;
  const int ZERO = P1;
  const double* cs = p.cs;
  const double2 z2 = make_double2(0.0, 0.0);
  if (TAB)
    for (int u = threadIdx.x; u < p.N2; u += blockDim.x) n2[u] = p.nu2_ab[u];
  const __amdgpu_buffer_rsrc_t r_me = raw_rsrc(p.me_col, p.n_me * 2);
  const __amdgpu_buffer_rsrc_t r_ch = raw_rsrc(p.ch_s, p.n_ch * 2);
  const __amdgpu_buffer_rsrc_t r_cs = raw_rsrc(cs, p.n_cs * (FOLD ? 16 : 8));
  for (int64_t e0 = (int64_t)blockIdx.x * NE; e0 < p.n_env; e0 += (int64_t)gridDim.x * NE) {
    // phase 0: one-particle values and adjoint accumulators
    for (int i = threadIdx.x; i < P1; i += blockDim.x) {
      const double leaf = GRAD ? re_w(load_coef<FOLD>(cs, p.cs_leaf + i)) : 0.0;
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        x[q][i] = e0 + q < p.n_env ? p.A[(e0 + q) * P1 + i] : z2;
        if (GRAD) ab[q].set(i, make_double2(leaf, 0.0));
      }
    }
    if (threadIdx.x == 0)
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        x[q][ZERO] = z2;
        if (GRAD) ab[q].set(ZERO, z2);
      }
    if (GRAD && FULL)
      for (int u = threadIdx.x; u < p.N2; u += blockDim.x)
#pragma unroll
        for (int q = 0; q < NE; ++q) ab[q].set(P1 + 1 + u, z2);
    __syncthreads();
    // phi = acc (unfolded); Re acc + i Im acci (folded)
    double2 acc[NE], acci[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) acc[q] = acci[q] = z2;
    // phase 1: the one-particle coefficients, and the order-2 values (an
    // invariant order-2 node's own term is an entry of the pair matrix, so
    // it has no coefficient here); four parent loads in flight per thread
    for (int i = threadIdx.x; i < P1; i += blockDim.x) {
      const RCoef<FOLD> k = load_coef<FOLD>(cs, p.cs_leaf + i);
#pragma unroll
      for (int q = 0; q < NE; ++q) coef_fma(k, x[q][i], acc[q], acci[q]);
    }
    for (int u0 = threadIdx.x; u0 < p.N2; u0 += 4 * blockDim.x) {
      uint32_t qq[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int u = u0 + r * (int)blockDim.x;
        qq[r] = u < p.N2 ? p.nu2_ab[u] : 0u;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int u = u0 + r * (int)blockDim.x;
        if (u < p.N2) {
          const int a = (int)(qq[r] & 0xffffu), b = (int)(qq[r] >> 16);
#pragma unroll
          for (int q = 0; q < NE; ++q) x[q][P1 + 1 + u] = cmul(x[q][a], x[q][b]);
        }
      }
    }
    __syncthreads();
    // phase 2a: resident-pair rows, y = M x (entry count padded to 4)
    for (int s = p.mr_wave[wid]; s < p.mr_wave[wid + 1]; ++s) {
      const int4 sl = p.mr_slice[s];
      const int row = p.mr_row[sl.x + lane];
      double2 y0[NE], y1[NE], y0i[NE], y1i[NE];
#pragma unroll
      for (int q = 0; q < NE; ++q) y0[q] = y1[q] = y0i[q] = y1i[q] = z2;
      const int z4 = sl.z & ~3;
      // entry column j of the slice: entry sl.y + 64 j + lane (wave-uniform part u)
      for (int j = z4; j < sl.z; ++j) {
        const int u = sl.y + j * 64;
        const int c0 = buf_u16(r_me, 2 * lane, 2 * u);
        const RCoef<FOLD> k0 = buf_coef<FOLD>(r_cs, lane, p.cs_me + u);
#pragma unroll
        for (int q = 0; q < NE; ++q) coef_fma(k0, x[q][c0], y0[q], y0i[q]);
      }
      for (int j = 0; j < z4; j += 4) {
        const int u = sl.y + j * 64;
        const int c0 = buf_u16(r_me, 2 * lane, 2 * u), c1 = buf_u16(r_me, 2 * lane, 2 * (u + 64));
        const int c2 = buf_u16(r_me, 2 * lane, 2 * (u + 128)), c3 = buf_u16(r_me, 2 * lane, 2 * (u + 192));
        const RCoef<FOLD> k0 = buf_coef<FOLD>(r_cs, lane, p.cs_me + u);
        const RCoef<FOLD> k1 = buf_coef<FOLD>(r_cs, lane, p.cs_me + u + 64);
        const RCoef<FOLD> k2 = buf_coef<FOLD>(r_cs, lane, p.cs_me + u + 128);
        const RCoef<FOLD> k3 = buf_coef<FOLD>(r_cs, lane, p.cs_me + u + 192);
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          const double2 x0 = x[q][c0], x1 = x[q][c1], x2 = x[q][c2], x3 = x[q][c3];
          coef_fma(k0, x0, y0[q], y0i[q]);
          coef_fma(k1, x1, y1[q], y1i[q]);
          coef_fma(k2, x2, y0[q], y0i[q]);
          coef_fma(k3, x3, y1[q], y1i[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const double2 y = make_double2(y0[q].x + y1[q].x, y0[q].y + y1[q].y);
        const double2 xr = x[q][row];
        const double2 h = cmul(xr, y);
        acc[q].x = fma(0.5, h.x, acc[q].x);
        acc[q].y = fma(0.5, h.y, acc[q].y);
        if (FOLD) {
          const double2 hi = cmul(xr, make_double2(y0i[q].x + y1i[q].x, y0i[q].y + y1i[q].y));
          acci[q].y = fma(0.5, hi.y, acci[q].y);
        }
        if (GRAD && row != ZERO) push_r<FULL>(P1, n2, x[q], ab[q], row, y);
      }
    }
    // phase 2b: trees.  Children whose sibling is one of the four hot slots
    // sit in fixed columns; their adjoint contributions are summed in
    // registers and pushed once per wave at the end.
    double2 xh0[NE], xh1[NE], xh2[NE], xh3[NE];
    double2 hacc0[NE], hacc1[NE], hacc2[NE], hacc3[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      xh0[q] = x[q][p.hot.x];
      xh1[q] = x[q][p.hot.y];
      xh2[q] = x[q][p.hot.z];
      xh3[q] = x[q][p.hot.w];
      hacc0[q] = hacc1[q] = hacc2[q] = hacc3[q] = z2;
    }
    for (int s = p.tr_wave[wid]; s < p.tr_wave[wid + 1]; ++s) {
      const int4 sl = p.tr_slice[s];
      const int item = sl.x + lane;
      const uint32_t qab = p.it_ab[item];
      const int a = (int)(qab & 0xffffu), b = (int)(qab >> 16);
      double2 xa[NE], xb[NE], xv[NE];
      // abar_v from childless children (t, and ti for Im phi when folded)
      double2 t[NE], ti[NE], asum[NE];   // asum: abar_v from children with children
      const RCoef<FOLD> kit = load_coef<FOLD>(cs, p.cs_it + item);
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        xa[q] = x[q][a];
        xb[q] = x[q][b];
        xv[q] = cmul(xa[q], xb[q]);
        t[q] = ti[q] = asum[q] = z2;
        coef_fma(kit, make_double2(1.0, 0.0), t[q], ti[q]);
      }
      {
        const int hp = p.cs_hot + item;
        const RCoef<FOLD> k0 = load_coef<FOLD>(cs, hp), k1 = load_coef<FOLD>(cs, hp + p.n_items);
        const RCoef<FOLD> k2 = load_coef<FOLD>(cs, hp + 2 * p.n_items), k3 = load_coef<FOLD>(cs, hp + 3 * p.n_items);
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          coef_fma(k0, xh0[q], t[q], ti[q]);
          coef_fma(k1, xh1[q], t[q], ti[q]);
          coef_fma(k2, xh2[q], t[q], ti[q]);
          coef_fma(k3, xh3[q], t[q], ti[q]);
          if (GRAD) {
            hacc0[q] = rfma(re_w(k0), xv[q], hacc0[q]);
            hacc1[q] = rfma(re_w(k1), xv[q], hacc1[q]);
            hacc2[q] = rfma(re_w(k2), xv[q], hacc2[q]);
            hacc3[q] = rfma(re_w(k3), xv[q], hacc3[q]);
          }
        }
      }
      const int cc = p.cs_ch;
      if (!GC) {
        // four children at a time, then the remainder (padding: sibling ZERO, coefficient 0)
        const int z4 = sl.z & ~3;
        for (int j = z4; j < sl.z; ++j) {
          const int u = sl.y + j * 64;
          const int s0 = buf_u16(r_ch, 2 * lane, 2 * u);
          const RCoef<FOLD> k0 = buf_coef<FOLD>(r_cs, lane, cc + u);
          const double r0 = re_w(k0);
#pragma unroll
          for (int q = 0; q < NE; ++q) {
            coef_fma(k0, x[q][s0], t[q], ti[q]);
            if (GRAD && r0 != 0.0) push_r<FULL>(P1, n2, x[q], ab[q], s0, make_double2(r0 * xv[q].x, r0 * xv[q].y));
          }
        }
        for (int j = 0; j < z4; j += 4) {
          const int u = sl.y + j * 64;
          const int s0 = buf_u16(r_ch, 2 * lane, 2 * u), s1 = buf_u16(r_ch, 2 * lane, 2 * (u + 64));
          const int s2 = buf_u16(r_ch, 2 * lane, 2 * (u + 128)), s3 = buf_u16(r_ch, 2 * lane, 2 * (u + 192));
          const RCoef<FOLD> k0 = buf_coef<FOLD>(r_cs, lane, cc + u), k1 = buf_coef<FOLD>(r_cs, lane, cc + u + 64);
          const RCoef<FOLD> k2 = buf_coef<FOLD>(r_cs, lane, cc + u + 128), k3 = buf_coef<FOLD>(r_cs, lane, cc + u + 192);
          const double r0 = re_w(k0), r1 = re_w(k1), r2 = re_w(k2), r3 = re_w(k3);
#pragma unroll
          for (int q = 0; q < NE; ++q) {
            const double2 x0 = x[q][s0], x1 = x[q][s1], x2 = x[q][s2], x3 = x[q][s3];
            coef_fma(k0, x0, t[q], ti[q]);
            coef_fma(k1, x1, t[q], ti[q]);
            coef_fma(k2, x2, t[q], ti[q]);
            coef_fma(k3, x3, t[q], ti[q]);
            if (GRAD) {
              const double2 v = xv[q];
              if (r0 != 0.0) push_r<FULL>(P1, n2, x[q], ab[q], s0, make_double2(r0 * v.x, r0 * v.y));
              if (r1 != 0.0) push_r<FULL>(P1, n2, x[q], ab[q], s1, make_double2(r1 * v.x, r1 * v.y));
              if (r2 != 0.0) push_r<FULL>(P1, n2, x[q], ab[q], s2, make_double2(r2 * v.x, r2 * v.y));
              if (r3 != 0.0) push_r<FULL>(P1, n2, x[q], ab[q], s3, make_double2(r3 * v.x, r3 * v.y));
            }
          }
        }
      } else {
        for (int j = 0; j < sl.z; ++j) {
          const int pos = sl.y + j * 64 + lane;
          const int sidx = p.ch_s[pos];
          const RCoef<FOLD> k = load_coef<FOLD>(cs, cc + pos);
          const double c = re_w(k);
          const int2 g = p.ch_g[pos];
          if (g.x == g.y) {
#pragma unroll
            for (int q = 0; q < NE; ++q) {
              coef_fma(k, x[q][sidx], t[q], ti[q]);
              if (GRAD && c != 0.0)
                push_r<FULL>(P1, n2, x[q], ab[q], sidx, make_double2(c * xv[q].x, c * xv[q].y));
            }
          } else {
            double2 xs[NE], xw[NE], aw[NE], awi[NE];
#pragma unroll
            for (int q = 0; q < NE; ++q) {
              xs[q] = x[q][sidx];
              xw[q] = cmul(xv[q], xs[q]);
              aw[q] = awi[q] = z2;
              coef_fma(k, make_double2(1.0, 0.0), aw[q], awi[q]);
            }
            for (int kk = g.x; kk < g.y; ++kk) {
              const int sg = p.gc_s[kk];
              const RCoef<FOLD> kg = load_coef<FOLD>(cs, p.cs_gc + kk);
              const double cg = re_w(kg);
#pragma unroll
              for (int q = 0; q < NE; ++q) {
                coef_fma(kg, x[q][sg], aw[q], awi[q]);
                if (GRAD) push_r<FULL>(P1, n2, x[q], ab[q], sg, make_double2(cg * xw[q].x, cg * xw[q].y));
              }
            }
#pragma unroll
            for (int q = 0; q < NE; ++q) {
              acc[q] = cfma(xw[q], aw[q], acc[q]);
              if (FOLD) acci[q] = cfma(xw[q], awi[q], acci[q]);
              if (GRAD) {
                push_r<FULL>(P1, n2, x[q], ab[q], sidx, cmul(aw[q], xv[q]));
                asum[q] = cfma(aw[q], xs[q], asum[q]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        acc[q] = cfma(xv[q], t[q], acc[q]);
        if (FOLD) acci[q] = cfma(xv[q], ti[q], acci[q]);
        if (GRAD && qab != ((uint32_t)ZERO | ((uint32_t)ZERO << 16))) {
          const double2 av = make_double2(t[q].x + asum[q].x, t[q].y + asum[q].y);
          push_r<FULL>(P1, n2, x[q], ab[q], a, cmul(av, xb[q]));
          push_r<FULL>(P1, n2, x[q], ab[q], b, cmul(av, xa[q]));
        }
      }
    }
    if (GRAD) {
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const double2 h0 = wave_sum(hacc0[q]), h1 = wave_sum(hacc1[q]);
        const double2 h2 = wave_sum(hacc2[q]), h3 = wave_sum(hacc3[q]);
        if (lane == 0) {
          if (p.hot.x != ZERO) push_r<FULL>(P1, n2, x[q], ab[q], p.hot.x, h0);
          if (p.hot.y != ZERO) push_r<FULL>(P1, n2, x[q], ab[q], p.hot.y, h1);
          if (p.hot.z != ZERO) push_r<FULL>(P1, n2, x[q], ab[q], p.hot.z, h2);
          if (p.hot.w != ZERO) push_r<FULL>(P1, n2, x[q], ab[q], p.hot.w, h3);
        }
      }
    }
    __syncthreads();
    if (GRAD && FULL) {
      // order-2 adjoints to the one-particle adjoints, abar_a += abar_u x_b, in
      // chunks of kForwardChunk entries per lane (a one-particle node can be
      // a parent of hundreds of order-2 nodes; padding entries name the zero
      // slot); all of a chunk's entries are loaded at once, the chunk sums are
      // added atomically, and no order-2 adjoint changes in this phase
      static_assert(kForwardChunk == 8, "two 16-byte entry loads per chunk");
      for (int c = threadIdx.x; c < p.n_fwck; c += blockDim.x) {
        const int tgt = p.fw_ck[c].x;
        const uint4* e4 = reinterpret_cast<const uint4*>(p.fw_ent + (size_t)c * kForwardChunk);
        const uint4 ea = e4[0], eb = e4[1];
        const uint32_t en[kForwardChunk] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
        double2 s2[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) s2[q] = z2;
#pragma unroll
        for (int f = 0; f < kForwardChunk; ++f)
#pragma unroll
          for (int q = 0; q < NE; ++q) s2[q] = cfma(ab[q].get(en[f] & 0xffffu), x[q][en[f] >> 16], s2[q]);
#pragma unroll
        for (int q = 0; q < NE; ++q) ab[q].add(tgt, s2[q]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      if (FOLD) acc[q].y = acci[q].y;
      const double2 phi = block_sum(acc[q], red);
      if (threadIdx.x == 0 && e0 + q < p.n_env) p.phi[e0 + q] = phi;
    }
    if (GRAD)
#pragma unroll
      for (int q = 0; q < NE; ++q)
        if (e0 + q < p.n_env) {
          double2* Be = p.Abar + (e0 + q) * P1;
          for (int i = threadIdx.x; i < P1; i += blockDim.x) Be[i] = ab[q].get(i);
        }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Rematerialising kernel, for DAGs whose resident set does not fit in LDS.
//
// Only the one-particle values A and adjoints Abar of one environment are
// resident (LDS).  Every term c_k x_k, k in K, is still the product of the
// two parents its DAG node names (Sec. 2.6), but the parents are recomputed
// from their one-particle factors instead of being stored.  Terms are
// grouped into rows keyed by a parent p ("row"); a lane item is a chunk of
// one row, y = sum_j M_j x_other_j, with every other parent of the chunk of
// the same order.
//   forward only: each term sits in the row of one parent, M = c, and
//                 phi += x_p y;
//   with adjoint: the terms form the symmetric matrix M over parents
//                 (M_pq = M_qp = c, M_pp = 2c), each term sits in the rows
//                 of both parents, phi += x_p y / 2 and abar_p = y exactly,
//                 so no adjoint is scattered per term.
// Factor lists hold LDS byte offsets of 16-byte slots (so the slots must
// number at most 4096).  The factors of the other parents may be
// precomputed products of two
// one-particle values (pair slots, filled in LDS per environment), which
// saves a read and a product per pair; row factors are one-particle slots.
// abar_p reaches the one-particle factors of p as y prod_{j != i} x_j
// (prefix and suffix products): one push per factor and item, with the
// four hottest one-particle slots summed in registers and pushed once per
// wave.  The rest are LDS atomics, so the reverse pass is not bitwise
// deterministic (the forward pass is).
//
// Folded schedules (FOLD) serve A with A_{n,l,-m} = (-1)^m conj(A_{n,l,m}),
// as the basis kernel produces: then x_kbar = conj(x_k) for the tuple kbar
// with every m negated, and a conjugate pair contributes
// (c_k + c_kbar) Re x_k + i (c_k - c_kbar) Im x_k to phi.  Only one tuple
// of each pair is evaluated; the adjoint of the real part uses the Re
// weight, which gives d Re(phi)/dA in the form Re sum_i abar_i dA_i (the
// adjoint itself differs from the unfolded one).
// ---------------------------------------------------------------------------
// d added to abar_s: in the register accumulator of s if s is one of the
// NH hot slots, else atomically in LDS (every index into h is a constant).
template <int K, int NH>
__device__ __forceinline__ void push_hot_from(const AdjPlanes& ab, int s, double2 d, const int4& hot,
                                              double2 (&h)[NH]) {
  if constexpr (K < NH) {
    const int hk = K == 0 ? hot.x : K == 1 ? hot.y : K == 2 ? hot.z : hot.w;
    if (s == hk) {
      h[K].x += d.x;
      h[K].y += d.y;
    } else {
      push_hot_from<K + 1, NH>(ab, s, d, hot, h);
    }
  } else {
    ab.add(s, d);
  }
}
template <int NH>
__device__ __forceinline__ void push_hot(const AdjPlanes& ab, int s, double2 d, const int4& hot, double2 (&h)[NH]) {
  push_hot_from<0, NH>(ab, s, d, hot, h);
}

// Field i of a packed factor list: the LDS byte offset of a 16-byte slot.
__device__ __forceinline__ int slot16(uint64_t lo, uint64_t hi, int i) {
  return (int)(((i < 4 ? lo : hi) >> (16 * (i & 3))) & 0xffffu);
}
__device__ __forceinline__ double2 lds_at(const double2* base, int byte_off) {
  return *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(base) + byte_off);
}

// value of one packed factor list of SIG factors
template <int SIG>
__device__ __forceinline__ double2 factor_product(const double2* x, uint64_t lo, uint64_t hi) {
  double2 v = lds_at(x, slot16(lo, hi, 0));
#pragma unroll
  for (int u = 1; u < SIG; ++u) v = cmul(v, lds_at(x, slot16(lo, hi, u)));
  return v;
}

// One lane item is a chunk of a row: the terms that share one parent (the
// row's base, a product of NB one-particle values) for NE environments,
// which share every metadata and coefficient load; environment e's values
// and adjoints sit xs and as double2 slots after those of environment e - 1.
//
// remat_entries: y1 = sum_j c'_j x_j (and y2 = sum_j c''_j x_j when
// folded) over the item's entries, x_j the other parent of term j, a
// product of SIG factors (one-particle values or pair products).
template <int SIG, bool FOLD, int NE>
__device__ __forceinline__ void remat_entries(const RematArgs& p, const EntryBufs& eb, const double2* x, int xs,
                                              const int4& sl, int lane, double2 (&y1)[NE], double2 (&y2)[NE]) {
  // entry metadata of this slice, prefetched one entry ahead of its use in
  // two register sets (the loop is unrolled by two); entry column j of the
  // slice sits at entry index sl.y + 64 j + lane
  const int vo = lane * 8;
  const int c0 = p.cs_ent + sl.y;   // wave-uniform coefficient index of column 0, lane 0
  const int n = sl.z;
#pragma unroll
  for (int e = 0; e < NE; ++e) y1[e] = y2[e] = make_double2(0.0, 0.0);
  if constexpr (NE > 1 && SIG > 4) {
    // long products of several environments: one entry in flight (registers)
    for (int j = 0; j < n; ++j) {
      const int so = (sl.y + 64 * j) * 8;
      const uint64_t lo = buf_u64(eb.lo, vo, so), hi = buf_u64(eb.hi, vo, so);
      const RCoef<FOLD> c = buf_coef<FOLD>(eb.cs, lane, c0 + 64 * j);
#pragma unroll
      for (int e = 0; e < NE; ++e) coef_fma<FOLD>(c, factor_product<SIG>(x + e * xs, lo, hi), y1[e], y2[e]);
    }
    return;
  }
  uint64_t a_lo = 0, a_hi = 0, b_lo = 0, b_hi = 0;
  RCoef<FOLD> a_c{}, b_c{};
  if (n > 0) {
    a_lo = buf_u64(eb.lo, vo, sl.y * 8);
    if (SIG > 4) a_hi = buf_u64(eb.hi, vo, sl.y * 8);
    a_c = buf_coef<FOLD>(eb.cs, lane, c0);
  }
  int j = 0;
  for (; j + 1 < n; j += 2) {
    const int so1 = (sl.y + 64 * (j + 1)) * 8;
    b_lo = buf_u64(eb.lo, vo, so1);
    if (SIG > 4) b_hi = buf_u64(eb.hi, vo, so1);
    b_c = buf_coef<FOLD>(eb.cs, lane, c0 + 64 * (j + 1));
#pragma unroll
    for (int e = 0; e < NE; ++e) coef_fma<FOLD>(a_c, factor_product<SIG>(x + e * xs, a_lo, a_hi), y1[e], y2[e]);
    if (j + 2 < n) {
      const int so2 = (sl.y + 64 * (j + 2)) * 8;
      a_lo = buf_u64(eb.lo, vo, so2);
      if (SIG > 4) a_hi = buf_u64(eb.hi, vo, so2);
      a_c = buf_coef<FOLD>(eb.cs, lane, c0 + 64 * (j + 2));
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) coef_fma<FOLD>(b_c, factor_product<SIG>(x + e * xs, b_lo, b_hi), y1[e], y2[e]);
  }
  if (j < n) {
#pragma unroll
    for (int e = 0; e < NE; ++e) coef_fma<FOLD>(a_c, factor_product<SIG>(x + e * xs, a_lo, a_hi), y1[e], y2[e]);
  }
}

// remat_row: the row value x_b (product of the NB row factors, whose
// packed offsets blo, bhi were loaded before the entries; the values are
// read after them so that they hold no registers there, and rows of up to
// five factors keep them for the suffix products), phi += x_b y
// (halved with the adjoint: every term sits in two rows), and with GRAD the
// adjoint y pushed to the row's factors by prefix and suffix products.  NH
// hot one-particle slots per environment are summed in registers.
template <bool GRAD, int NB, bool FOLD, int NE, int NH>
__device__ __forceinline__ void remat_row(const RematArgs& p, const double2* x, double* ab, int xs, int as,
                                          uint64_t blo, uint64_t bhi, const double2 (&y1)[NE],
                                          const double2 (&y2)[NE], double2 (&acc)[NE], double2 (&hot)[NE][NH]) {
  const double w = GRAD ? 0.5 : 1.0;
  const bool push = GRAD && slot16(blo, bhi, 0) != 16 * p.P1;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const double2* xe = x + e * xs;
    constexpr bool KEEP = NB <= 5;   // factor values kept in registers for the suffix products
    double2 pre[NB], xf[KEEP ? NB : 1];
    if constexpr (KEEP) {
#pragma unroll
      for (int i = 0; i < NB; ++i) xf[i] = lds_at(xe, slot16(blo, bhi, i));
    } else {
      xf[0] = lds_at(xe, slot16(blo, bhi, 0));
    }
    double2 xb = xf[0];
    pre[0] = make_double2(1.0, 0.0);
#pragma unroll
    for (int i = 1; i < NB; ++i) {
      pre[i] = xb;
      if constexpr (KEEP)
        xb = cmul(xb, xf[i]);
      else
        xb = cmul(xb, lds_at(xe, slot16(blo, bhi, i)));
    }
    if constexpr (FOLD) {
      acc[e].x = fma(w, xb.x * y1[e].x - xb.y * y1[e].y, acc[e].x);
      acc[e].y = fma(w, xb.x * y2[e].y + xb.y * y2[e].x, acc[e].y);
    } else {
      const double2 h = cmul(xb, y1[e]);
      acc[e].x = fma(w, h.x, acc[e].x);
      acc[e].y = fma(w, h.y, acc[e].y);
    }
    if (push) {
      double2 suf = y1[e];
#pragma unroll
      for (int i = NB - 1; i >= 0; --i) {
        push_hot<NH>(AdjPlanes{ab + 2 * e * as, as}, slot16(blo, bhi, i) >> 4, i == 0 ? suf : cmul(pre[i], suf),
                     p.hot, hot[e]);
        if (i > 0) {
          if constexpr (KEEP)
            suf = cmul(suf, xf[i]);
          else
            suf = cmul(suf, lds_at(xe, slot16(blo, bhi, i)));
        }
      }
    }
  }
}

constexpr int kRematBlock = 1024;

// NE environments per block (1 or 2): the block's slices are walked once,
// each lane item evaluating its terms for every environment of the block
// from the same metadata; a missing last environment computes on zeros and
// writes nothing.  BIG: blocks of up to 1024 threads (at most 128 VGPRs),
// else up to 512.
template <bool GRAD, bool FOLD, int NE, bool BIG>
__global__ __launch_bounds__(BIG ? kRematBlock : kRematBlock / 2) void remat_kernel(RematArgs p) {
  constexpr int NH = NE == 1 ? 4 : 2;
  extern __shared__ double2 lds[];
  const int P1 = p.P1;
  const int ONE = P1;
  const int xs = P1 + 1 + p.n_pairs;   // values per environment: one-particle, constant one, pair products
  const int as = GRAD ? P1 + 1 : 0;    // one-particle adjoints per environment
  double2* x = lds;                    // [NE][xs]
  double* ab = reinterpret_cast<double*>(lds + NE * xs);   // [NE][2][as]: Re and Im planes (AdjPlanes)
  double2* red = reinterpret_cast<double2*>(ab + 2 * NE * as);
  const int lane = threadIdx.x & 63;
  // wave index, made visibly uniform so that slice descriptors and loop
  // bounds live in scalar registers
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const EntryBufs eb{raw_rsrc(p.oth_lo, p.n_ent * 8), raw_rsrc(p.oth_hi, p.n_ent * 8),
                     raw_rsrc(p.cs, (p.cs_ent + p.n_ent) * (FOLD ? 16 : 8))};
  for (int64_t e0 = (int64_t)blockIdx.x * NE; e0 < p.n_env; e0 += (int64_t)gridDim.x * NE) {
    const int ne = (int)min((int64_t)NE, p.n_env - e0);
    double2 acc[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) acc[e] = make_double2(0.0, 0.0);
    for (int i = threadIdx.x; i < P1; i += blockDim.x) {
      const RCoef<FOLD> k = load_coef<FOLD>(p.cs, (unsigned)(p.cs_leaf + i));
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const double2 a = e < ne ? p.A[(e0 + e) * P1 + i] : make_double2(0.0, 0.0);
        x[e * xs + i] = a;
        if constexpr (FOLD) {
          if (GRAD) {
            ab[2 * e * as + i] = k.c.x;
            ab[(2 * e + 1) * as + i] = 0.0;
          }
          acc[e].x = fma(k.c.x, a.x, acc[e].x);
          acc[e].y = fma(k.c.y, a.y, acc[e].y);
        } else {
          if (GRAD) {
            ab[2 * e * as + i] = k.c;
            ab[(2 * e + 1) * as + i] = 0.0;
          }
          acc[e] = rfma(k.c, a, acc[e]);
        }
      }
    }
    if (threadIdx.x < NE) {
      x[threadIdx.x * xs + ONE] = make_double2(1.0, 0.0);
      if (GRAD) ab[2 * threadIdx.x * as + ONE] = ab[(2 * threadIdx.x + 1) * as + ONE] = 0.0;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < p.n_pairs; r += blockDim.x) {
      const uint32_t q = p.pairs[r];
#pragma unroll
      for (int e = 0; e < NE; ++e) x[e * xs + ONE + 1 + r] = cmul(x[e * xs + (q & 0xffffu)], x[e * xs + (q >> 16)]);
    }
    __syncthreads();
    double2 hot[NE][NH];
#pragma unroll
    for (int e = 0; e < NE; ++e)
#pragma unroll
      for (int h = 0; h < NH; ++h) hot[e][h] = make_double2(0.0, 0.0);
    for (int s = wid; s < p.n_slices; s += nw) {
      const int4 sl = p.slice[s];
      // the row's factor offsets, loaded ahead of the entries
      const int item = sl.x + lane;
      const uint64_t blo = p.row_lo[item];
      const uint64_t bhi = (sl.w & 0xff) > 4 ? p.row_hi[item] : 0;
      double2 y1[NE], y2[NE];
      switch (sl.w >> 8) {
        case 1: remat_entries<1, FOLD, NE>(p, eb, x, xs, sl, lane, y1, y2); break;
        case 2: remat_entries<2, FOLD, NE>(p, eb, x, xs, sl, lane, y1, y2); break;
        case 3: remat_entries<3, FOLD, NE>(p, eb, x, xs, sl, lane, y1, y2); break;
        case 4: remat_entries<4, FOLD, NE>(p, eb, x, xs, sl, lane, y1, y2); break;
        case 5: remat_entries<5, FOLD, NE>(p, eb, x, xs, sl, lane, y1, y2); break;
        case 6: remat_entries<6, FOLD, NE>(p, eb, x, xs, sl, lane, y1, y2); break;
        default: remat_entries<7, FOLD, NE>(p, eb, x, xs, sl, lane, y1, y2); break;
      }
      switch (sl.w & 0xff) {
        case 1: remat_row<GRAD, 1, FOLD, NE, NH>(p, x, ab, xs, as, blo, bhi, y1, y2, acc, hot); break;
        case 2: remat_row<GRAD, 2, FOLD, NE, NH>(p, x, ab, xs, as, blo, bhi, y1, y2, acc, hot); break;
        case 3: remat_row<GRAD, 3, FOLD, NE, NH>(p, x, ab, xs, as, blo, bhi, y1, y2, acc, hot); break;
        case 4: remat_row<GRAD, 4, FOLD, NE, NH>(p, x, ab, xs, as, blo, bhi, y1, y2, acc, hot); break;
        case 5: remat_row<GRAD, 5, FOLD, NE, NH>(p, x, ab, xs, as, blo, bhi, y1, y2, acc, hot); break;
        case 6: remat_row<GRAD, 6, FOLD, NE, NH>(p, x, ab, xs, as, blo, bhi, y1, y2, acc, hot); break;
        case 7: remat_row<GRAD, 7, FOLD, NE, NH>(p, x, ab, xs, as, blo, bhi, y1, y2, acc, hot); break;
        default: remat_row<GRAD, 8, FOLD, NE, NH>(p, x, ab, xs, as, blo, bhi, y1, y2, acc, hot); break;
      }
    }
    if (GRAD) {
      const int hs[4] = {p.hot.x, p.hot.y, p.hot.z, p.hot.w};
#pragma unroll
      for (int e = 0; e < NE; ++e)
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const double2 v = wave_sum(hot[e][h]);
          if (lane == 0 && hs[h] != ONE) AdjPlanes{ab + 2 * e * as, as}.add(hs[h], v);
        }
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const double2 phi = block_sum(acc[e], red);   // synchronises the block
      if (threadIdx.x == 0 && e < ne) p.phi[e0 + e] = phi;
    }
    if (GRAD) {
      for (int e = 0; e < ne; ++e) {
        double2* Be = p.Abar + (e0 + e) * P1;
        for (int i = threadIdx.x; i < P1; i += blockDim.x)
          Be[i] = make_double2(ab[2 * e * as + i], ab[(2 * e + 1) * as + i]);
      }
    }
    __syncthreads();
  }
}

template __global__ void remat_kernel<false, false, 1, false>(RematArgs);
template __global__ void remat_kernel<true, false, 1, false>(RematArgs);
template __global__ void remat_kernel<false, true, 1, false>(RematArgs);
template __global__ void remat_kernel<true, true, 1, false>(RematArgs);
template __global__ void remat_kernel<false, false, 2, false>(RematArgs);
template __global__ void remat_kernel<true, false, 2, false>(RematArgs);
template __global__ void remat_kernel<false, true, 2, false>(RematArgs);
template __global__ void remat_kernel<true, true, 2, false>(RematArgs);
template __global__ void remat_kernel<false, false, 1, true>(RematArgs);
template __global__ void remat_kernel<true, false, 1, true>(RematArgs);
template __global__ void remat_kernel<false, true, 1, true>(RematArgs);
template __global__ void remat_kernel<true, true, 1, true>(RematArgs);
template __global__ void remat_kernel<false, false, 2, true>(RematArgs);
template __global__ void remat_kernel<true, false, 2, true>(RematArgs);
template __global__ void remat_kernel<false, true, 2, true>(RematArgs);
template __global__ void remat_kernel<true, true, 2, true>(RematArgs);

__global__ __launch_bounds__(256) void prep_fold_kernel(PrepFoldArgs p) {
  prep_fold_range(p, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

template __global__ void forest_kernel<false, false, false, false, 1>(ForestArgs);
template __global__ void forest_kernel<false, true, false, false, 1>(ForestArgs);
template __global__ void forest_kernel<true, false, false, false, 1>(ForestArgs);
template __global__ void forest_kernel<true, true, false, false, 1>(ForestArgs);
template __global__ void forest_kernel<true, false, true, false, 1>(ForestArgs);
template __global__ void forest_kernel<true, true, true, false, 1>(ForestArgs);
template __global__ void forest_kernel<false, false, false, true, 1>(ForestArgs);
template __global__ void forest_kernel<false, true, false, true, 1>(ForestArgs);
template __global__ void forest_kernel<true, false, false, true, 1>(ForestArgs);
template __global__ void forest_kernel<true, true, false, true, 1>(ForestArgs);
template __global__ void forest_kernel<true, false, true, true, 1>(ForestArgs);
template __global__ void forest_kernel<true, true, true, true, 1>(ForestArgs);
template __global__ void forest_kernel<false, false, false, false, 2>(ForestArgs);
template __global__ void forest_kernel<false, true, false, false, 2>(ForestArgs);
template __global__ void forest_kernel<true, false, false, false, 2>(ForestArgs);
template __global__ void forest_kernel<true, true, false, false, 2>(ForestArgs);
template __global__ void forest_kernel<true, false, true, false, 2>(ForestArgs);
template __global__ void forest_kernel<true, true, true, false, 2>(ForestArgs);
template __global__ void forest_kernel<false, false, false, true, 2>(ForestArgs);
template __global__ void forest_kernel<false, true, false, true, 2>(ForestArgs);
template __global__ void forest_kernel<true, false, false, true, 2>(ForestArgs);
template __global__ void forest_kernel<true, true, false, true, 2>(ForestArgs);
template __global__ void forest_kernel<true, false, true, true, 2>(ForestArgs);
template __global__ void forest_kernel<true, true, true, true, 2>(ForestArgs);

}  // namespace ace
