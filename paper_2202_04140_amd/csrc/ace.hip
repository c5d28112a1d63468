// C ABI of the evaluator (declared in include/ace.h): graph build and
// upload, workspace sizing, and the launch sequences of ace_basis,
// ace_contract, ace_eval and ace_eval_grad.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ace.h"
#include "ace_kernels.hpp"
#include "graph.hpp"
// the kernels are compiled in this translation unit
#include "kernels.hip"

namespace ace {
namespace {

thread_local std::string g_error;

ace_status fail(ace_status code, const std::string& msg) {
  g_error = msg;
  return code;
}

#define ACE_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ACE_ERR_HIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kDagThreads = 256;
constexpr int kNaiveThreads = 256;
constexpr int kBasisThreads = 256;
constexpr int kGradThreads = 64;
constexpr int kArenaBlocks = 1024;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace
}  // namespace ace

using namespace ace;

// ---------------------------------------------------------------------------
// graph object
// ---------------------------------------------------------------------------
struct ace_graph {
  HostGraph h;
  ace_graph_stats stats{};
  bool on_device = false;
  int device = -1;
  // evaluation schedule (host copies)
  int P1 = 0, S = 0, T = 0, slots = 0, depth = 0;
  int st_off[kMaxLayers + 2] = {0};
  int cl_off[kMaxLayers + 2] = {0};
  std::vector<int2> st_ab, cl_ab;
  std::vector<int32_t> st_k, cl_k, leaf_k;
  std::vector<int16_t> naive_tup;
  std::vector<OnepInfo> onep;
  std::vector<int16_t> onep_index;
  std::vector<double> ycoef;
  // device copies (one allocation)
  void* dmem = nullptr;
  int2 *d_st_ab = nullptr, *d_cl_ab = nullptr;
  int32_t *d_st_k = nullptr, *d_cl_k = nullptr, *d_leaf_k = nullptr;
  int16_t *d_naive_tup = nullptr, *d_onep_index = nullptr;
  OnepInfo* d_onep = nullptr;
  double* d_ycoef = nullptr;
  // LDS plan
  size_t max_lds = 0;
  bool fwd_xl = false;    // forward-only: value arena in LDS
  bool grad_xl = false;   // forward+reverse: value arena in LDS
  bool grad_al = false;   // forward+reverse: adjoint arena in LDS
};

namespace {

// Normalised associated-Legendre recurrence coefficients for complex
// orthonormal Y_l^m with the Condon-Shortley phase (m >= 0):
//   q_m^m = (-1)^m K_mm (2m-1)!!,   K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
//   q_l^m = A_lm z q_{l-1}^m - B_lm q_{l-2}^m
//   A_lm = sqrt((4l^2-1)/(l^2-m^2)),
//   B_lm = sqrt((2l+1)((l-1)^2-m^2)/((2l-3)(l^2-m^2)))
void make_ycoef(int L, std::vector<double>& out) {
  const int NY = (L + 1) * (L + 2) / 2;
  out.assign(3 * NY, 0.0);
  for (int m = 0; m <= L; ++m) {
    // K_mm (2m-1)!! = sqrt((2m+1)/(4 pi) / (2m)!) (2m-1)!!
    long double v = 1.0L / (4.0L * 3.14159265358979323846264338327950288L);
    v *= (long double)(2 * m + 1);
    long double s = 1.0L;  // (2m-1)!!^2 / (2m)! = prod_{k=1}^{m} (2k-1)/(2k)
    for (int k = 1; k <= m; ++k) s *= (long double)(2 * k - 1) / (long double)(2 * k);
    long double start = std::sqrt(v * s);
    if (m & 1) start = -start;
    out[2 * NY + (m * (m + 1)) / 2 + m] = (double)start;
    for (int l = m + 1; l <= L; ++l) {
      const int o = (l * (l + 1)) / 2 + m;
      const long double ll = l, mm = m;
      out[o] = (double)std::sqrt((4.0L * ll * ll - 1.0L) / (ll * ll - mm * mm));
      if (l >= m + 2)
        out[NY + o] = (double)std::sqrt((2.0L * ll + 1.0L) * ((ll - 1.0L) * (ll - 1.0L) - mm * mm) /
                                        ((2.0L * ll - 3.0L) * (ll * ll - mm * mm)));
    }
  }
}

void make_schedule(ace_graph* g) {
  const HostGraph& h = g->h;
  const int64_t V = h.n_nodes();
  const int P1 = h.P1;
  g->P1 = P1;
  // liveness: a node matters if it is a tuple of K or has a live child.
  // Parents always precede children in insertion order.
  std::vector<uint8_t> live(V, 0);
  for (int64_t v = 0; v < V; ++v) live[v] = h.node_k[v] >= 0;
  std::vector<int32_t> live_children(V, 0);
  for (int64_t v = V - 1; v >= P1; --v) {
    if (!live[v]) continue;
    const int32_t a = h.par[2 * v], b = h.par[2 * v + 1];
    live[a] = 1;
    live[b] = 1;
    live_children[a] += 1;
    live_children[b] += 1;
  }
  // stored product nodes, ordered by (layer, id) -> slots P1..
  std::vector<std::vector<int32_t>> st_by_layer(h.depth + 1), cl_by_layer(h.depth + 1);
  for (int64_t v = P1; v < V; ++v) {
    if (!live[v]) continue;
    if (live_children[v] > 0)
      st_by_layer[h.layer[v]].push_back((int32_t)v);
    else
      cl_by_layer[h.layer[v]].push_back((int32_t)v);
  }
  if (h.depth > kMaxLayers) throw std::length_error("DAG deeper than supported");
  std::vector<int32_t> slot(V, -1);
  for (int i = 0; i < P1; ++i) slot[i] = i;
  int s = P1;
  for (int L = 1; L <= h.depth; ++L)
    for (int32_t v : st_by_layer[L]) slot[v] = s++;
  g->slots = s;
  g->S = s - P1;
  g->depth = h.depth;
  g->st_ab.clear();
  g->st_k.clear();
  g->cl_ab.clear();
  g->cl_k.clear();
  g->st_off[0] = g->st_off[1] = 0;
  g->cl_off[0] = g->cl_off[1] = 0;
  for (int L = 1; L <= h.depth; ++L) {
    g->st_off[L] = (int)g->st_ab.size();
    for (int32_t v : st_by_layer[L]) {
      g->st_ab.push_back(make_int2(slot[h.par[2 * v]], slot[h.par[2 * v + 1]]));
      g->st_k.push_back(h.node_k[v]);
    }
    g->cl_off[L] = (int)g->cl_ab.size();
    for (int32_t v : cl_by_layer[L]) {
      if (h.node_k[v] < 0) throw std::logic_error("childless auxiliary node survived liveness");
      g->cl_ab.push_back(make_int2(slot[h.par[2 * v]], slot[h.par[2 * v + 1]]));
      g->cl_k.push_back(h.node_k[v]);
    }
  }
  g->st_off[h.depth + 1] = (int)g->st_ab.size();
  g->cl_off[h.depth + 1] = (int)g->cl_ab.size();
  g->T = (int)g->cl_ab.size();
  g->leaf_k.assign(P1, -1);
  for (int i = 0; i < P1; ++i) g->leaf_k[i] = h.node_k[i];

  // naive tuples, padded with the constant-one slot P1
  if (P1 > 32766) throw std::length_error("too many one-particle functions for int16 tuples");
  g->naive_tup.assign((size_t)h.nK * h.width, (int16_t)P1);
  for (int64_t q = 0; q < h.nK; ++q)
    for (int t = 0; t < h.k_len[q]; ++t) g->naive_tup[(size_t)q * h.width + t] = (int16_t)h.k_flat[(size_t)q * h.width + t];

  // one-particle tables (O(3) only)
  g->onep.clear();
  g->onep_index.clear();
  g->ycoef.clear();
  if (h.spec.group == 0) {
    const int L = h.spec.l_max, N = h.spec.n_max, W = 2 * L + 1;
    g->onep_index.assign((size_t)(N + 1) * (L + 1) * W, (int16_t)-1);
    for (int i = 0; i < P1; ++i) {
      const int n = h.on_n[i], l = h.on_l[i], m = h.on_m[i];
      OnepInfo o{};
      o.n = (int16_t)n;
      const int am = m < 0 ? -m : m;
      o.yoff = (int16_t)((l * (l + 1)) / 2 + am);
      const int sgn = (am & 1) ? -1 : 1;
      o.sre = (int8_t)(m < 0 ? sgn : 1);
      o.sim = (int8_t)(m < 0 ? -sgn : 1);
      g->onep.push_back(o);
      g->onep_index[(size_t)(n * (L + 1) + l) * W + (m + L)] = (int16_t)i;
    }
    make_ycoef(L, g->ycoef);
  }
}

void make_stats(ace_graph* g) {
  const HostGraph& h = g->h;
  ace_graph_stats& st = g->stats;
  std::memset(&st, 0, sizeof(st));
  st.n_onep = h.P1;
  st.n_k = h.nK;
  for (int i = 0; i <= 8; ++i) st.n_k_by_order[i] = h.nK_by_order[i];
  st.n_nodes = h.n_nodes();
  for (int64_t v = h.P1; v < h.n_nodes(); ++v) {
    if (h.node_k[v] < 0) {
      st.n_aux += 1;
      st.n_aux_by_order[h.node_len[v]] += 1;
    }
    if (h.nchild[v] > 0)
      st.n_stored += 1;
    else
      st.n_childless += 1;
  }
  for (int i = 0; i < h.P1; ++i)
    if (h.nchild[i] > 0) st.n_leaf_parents += 1;
  st.depth = h.depth;
  for (int64_t v = 0; v < h.n_nodes(); ++v)
    if (h.layer[v] < 16) st.n_layer[h.layer[v]] += 1;
  for (int64_t q = 0; q < h.nK; ++q) st.naive_cmuls += h.k_len[q] - 1;
}

template <typename T>
T* carve(char*& p, size_t n) {
  T* r = reinterpret_cast<T*>(p);
  p += align_up(n * sizeof(T));
  return r;
}

ace_status upload(ace_graph* g) {
  int dev = 0;
  ACE_HIP(hipGetDevice(&dev));
  g->device = dev;
  int lds = 0;
  ACE_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  g->max_lds = (size_t)lds;
  size_t bytes = 0;
  bytes += align_up(g->st_ab.size() * sizeof(int2)) + align_up(g->st_k.size() * 4);
  bytes += align_up(g->cl_ab.size() * sizeof(int2)) + align_up(g->cl_k.size() * 4);
  bytes += align_up(g->leaf_k.size() * 4) + align_up(g->naive_tup.size() * 2);
  bytes += align_up(g->onep.size() * sizeof(OnepInfo)) + align_up(g->onep_index.size() * 2);
  bytes += align_up(g->ycoef.size() * 8) + kAlign;
  if (hipMalloc(&g->dmem, bytes) != hipSuccess) {
    g->dmem = nullptr;
    (void)hipGetLastError();
    return fail(ACE_ERR_OUT_OF_MEMORY, "hipMalloc of the graph schedule failed");
  }
  char* p = static_cast<char*>(g->dmem);
  g->d_st_ab = carve<int2>(p, g->st_ab.size());
  g->d_st_k = carve<int32_t>(p, g->st_k.size());
  g->d_cl_ab = carve<int2>(p, g->cl_ab.size());
  g->d_cl_k = carve<int32_t>(p, g->cl_k.size());
  g->d_leaf_k = carve<int32_t>(p, g->leaf_k.size());
  g->d_naive_tup = carve<int16_t>(p, g->naive_tup.size());
  g->d_onep = carve<OnepInfo>(p, g->onep.size());
  g->d_onep_index = carve<int16_t>(p, g->onep_index.size());
  g->d_ycoef = carve<double>(p, g->ycoef.size());
  auto put = [](void* d, const void* s, size_t n) { return n ? hipMemcpy(d, s, n, hipMemcpyHostToDevice) : hipSuccess; };
  ACE_HIP(put(g->d_st_ab, g->st_ab.data(), g->st_ab.size() * sizeof(int2)));
  ACE_HIP(put(g->d_st_k, g->st_k.data(), g->st_k.size() * 4));
  ACE_HIP(put(g->d_cl_ab, g->cl_ab.data(), g->cl_ab.size() * sizeof(int2)));
  ACE_HIP(put(g->d_cl_k, g->cl_k.data(), g->cl_k.size() * 4));
  ACE_HIP(put(g->d_leaf_k, g->leaf_k.data(), g->leaf_k.size() * 4));
  ACE_HIP(put(g->d_naive_tup, g->naive_tup.data(), g->naive_tup.size() * 2));
  ACE_HIP(put(g->d_onep, g->onep.data(), g->onep.size() * sizeof(OnepInfo)));
  ACE_HIP(put(g->d_onep_index, g->onep_index.data(), g->onep_index.size() * 2));
  ACE_HIP(put(g->d_ycoef, g->ycoef.data(), g->ycoef.size() * 8));

  // LDS plan for the DAG kernel
  const size_t red = (kDagThreads / 64) * sizeof(double2);
  const size_t arena = (size_t)g->slots * sizeof(double2);
  g->fwd_xl = arena + red <= g->max_lds;
  g->grad_xl = g->fwd_xl;
  g->grad_al = 2 * arena + red <= g->max_lds;
  const int maxl = (int)g->max_lds;
  ACE_HIP(hipFuncSetAttribute((const void*)dag_kernel<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  ACE_HIP(hipFuncSetAttribute((const void*)dag_kernel<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  ACE_HIP(hipFuncSetAttribute((const void*)dag_kernel<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  ACE_HIP(hipFuncSetAttribute((const void*)basis_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  ACE_HIP(hipFuncSetAttribute((const void*)grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  g->on_device = true;
  return ACE_OK;
}

bool valid_graph(const ace_graph* g) { return g != nullptr; }

ace_status need_device(const ace_graph* g) {
  if (!g) return fail(ACE_ERR_INVALID_ARG, "graph is NULL");
  if (!g->on_device) return fail(ACE_ERR_INVALID_ARG, "graph was built with ACE_BUILD_HOST_ONLY");
  if (g->h.spec.group != 0) return fail(ACE_ERR_UNSUPPORTED, "evaluation is implemented for the O(3) basis only");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != g->device)
    return fail(ACE_ERR_INVALID_ARG, "graph belongs to another HIP device than the current one");
  return ACE_OK;
}

// workspace layout for n_env environments
struct Workspace {
  double2* A = nullptr;
  double2* Abar = nullptr;
  double2* arena_x = nullptr;
  double2* arena_ab = nullptr;
  size_t bytes = 0;
};

int arena_blocks(int64_t n_env) { return (int)std::max<int64_t>(1, std::min<int64_t>(n_env, kArenaBlocks)); }

Workspace plan_workspace(const ace_graph* g, int64_t n_env, char* base) {
  Workspace w;
  size_t off = 0;
  auto take = [&](size_t n) {
    char* r = base ? base + off : nullptr;
    off += align_up(n);
    return reinterpret_cast<double2*>(r);
  };
  const size_t per_env = (size_t)g->P1 * sizeof(double2);
  w.A = take((size_t)n_env * per_env);
  w.Abar = take((size_t)n_env * per_env);
  const size_t arena = (size_t)arena_blocks(n_env) * g->slots * sizeof(double2);
  if (!g->fwd_xl || !g->grad_xl) w.arena_x = take(arena);
  if (!g->grad_al) w.arena_ab = take(arena);
  w.bytes = off;
  return w;
}

ace_status check_offsets(const int32_t* offsets, int64_t n_env, int64_t n_nbr, hipStream_t s) {
  std::vector<int32_t> h((size_t)n_env + 1);
  ACE_HIP(hipMemcpyAsync(h.data(), offsets, h.size() * 4, hipMemcpyDeviceToHost, s));
  ACE_HIP(hipStreamSynchronize(s));
  if (h[0] != 0) return fail(ACE_ERR_INVALID_ARG, "offsets[0] must be 0");
  for (int64_t e = 0; e < n_env; ++e)
    if (h[e + 1] < h[e]) return fail(ACE_ERR_INVALID_ARG, "offsets must be non-decreasing");
  if (n_nbr >= 0 && h[n_env] != n_nbr) return fail(ACE_ERR_INVALID_ARG, "offsets[n_env] must equal n_nbr");
  return ACE_OK;
}

int64_t grid_for(int64_t n_env) { return std::max<int64_t>(1, std::min<int64_t>(n_env, (int64_t)1 << 30)); }

ace_status launch_basis(const ace_graph* g, int64_t n_env, const int32_t* offsets, const double* pos, double2* A,
                        hipStream_t s) {
  BasisArgs a{};
  a.n_env = n_env;
  a.offsets = offsets;
  a.pos = pos;
  a.A = A;
  a.onep = g->d_onep;
  a.ycoef = g->d_ycoef;
  a.P1 = g->P1;
  a.n_max = g->h.spec.n_max;
  a.l_max = g->h.spec.l_max;
  a.r_cut = g->h.spec.r_cut;
  const int NY = (a.l_max + 1) * (a.l_max + 2) / 2;
  const size_t lds = (size_t)g->P1 * 16 + (size_t)32 * ((a.n_max + 1) + 2 * NY) * 8;
  if (lds > g->max_lds) return fail(ACE_ERR_UNSUPPORTED, "one-particle basis too large for the basis kernel");
  hipLaunchKernelGGL(basis_kernel, dim3((unsigned)grid_for(n_env)), dim3(kBasisThreads), lds, s, a);
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

ace_status launch_dag(const ace_graph* g, const double* coeffs, int64_t n_env, const double2* A, double2* phi,
                      double2* Abar, const Workspace& w, hipStream_t s) {
  DagArgs a{};
  a.n_env = n_env;
  a.A = A;
  a.phi = phi;
  a.Abar = Abar;
  a.coeffs = coeffs;
  a.st_ab = g->d_st_ab;
  a.st_k = g->d_st_k;
  a.cl_ab = g->d_cl_ab;
  a.cl_k = g->d_cl_k;
  a.leaf_k = g->d_leaf_k;
  a.arena_x = w.arena_x;
  a.arena_ab = w.arena_ab;
  a.P1 = g->P1;
  a.S = g->S;
  a.slots = g->slots;
  a.depth = g->depth;
  std::memcpy(a.st_off, g->st_off, sizeof(a.st_off));
  std::memcpy(a.cl_off, g->cl_off, sizeof(a.cl_off));
  const size_t red = (kDagThreads / 64) * sizeof(double2);
  const size_t arena = (size_t)g->slots * sizeof(double2);
  const bool grad = Abar != nullptr;
  // Variant, LDS bytes and grid.  A global arena is indexed by block, so
  // every variant that touches one runs on arena_blocks() blocks (the
  // workspace holds that many arenas); the rest get one block per env.
  const dim3 block(kDagThreads);
  if (!grad) {
    if (g->fwd_xl)
      hipLaunchKernelGGL((dag_kernel<true, false>), dim3((unsigned)grid_for(n_env)), block, red + arena, s, a);
    else
      hipLaunchKernelGGL((dag_kernel<false, false>), dim3((unsigned)arena_blocks(n_env)), block, red, s, a);
  } else if (g->grad_xl && g->grad_al) {
    hipLaunchKernelGGL((dag_kernel<true, true>), dim3((unsigned)grid_for(n_env)), block, red + 2 * arena, s, a);
  } else if (g->grad_xl) {
    hipLaunchKernelGGL((dag_kernel<true, false>), dim3((unsigned)arena_blocks(n_env)), block, red + arena, s, a);
  } else {
    hipLaunchKernelGGL((dag_kernel<false, false>), dim3((unsigned)arena_blocks(n_env)), block, red, s, a);
  }
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

ace_status launch_naive(const ace_graph* g, const double* coeffs, int64_t n_env, const double2* A, double2* phi,
                        double2* Abar, hipStream_t s) {
  NaiveArgs a{};
  a.n_env = n_env;
  a.A = A;
  a.phi = phi;
  a.Abar = Abar;
  a.coeffs = coeffs;
  a.tup = g->d_naive_tup;
  a.nK = g->h.nK;
  a.P1 = g->P1;
  a.nu_max = g->h.width;
  const size_t lds = (size_t)(2 * (g->P1 + 1) + kNaiveThreads / 64) * sizeof(double2);
  if (lds > g->max_lds) return fail(ACE_ERR_UNSUPPORTED, "one-particle basis too large for the naive kernel");
  const dim3 grid((unsigned)grid_for(n_env)), block(kNaiveThreads);
  switch (a.nu_max) {
    case 1: hipLaunchKernelGGL(naive_kernel<1>, grid, block, lds, s, a); break;
    case 2: hipLaunchKernelGGL(naive_kernel<2>, grid, block, lds, s, a); break;
    case 3: hipLaunchKernelGGL(naive_kernel<3>, grid, block, lds, s, a); break;
    case 4: hipLaunchKernelGGL(naive_kernel<4>, grid, block, lds, s, a); break;
    case 5: hipLaunchKernelGGL(naive_kernel<5>, grid, block, lds, s, a); break;
    case 6: hipLaunchKernelGGL(naive_kernel<6>, grid, block, lds, s, a); break;
    case 7: hipLaunchKernelGGL(naive_kernel<7>, grid, block, lds, s, a); break;
    default: hipLaunchKernelGGL(naive_kernel<8>, grid, block, lds, s, a); break;
  }
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

ace_status launch_grad(const ace_graph* g, int64_t n_env, const int32_t* offsets, const double* pos,
                       const double2* Abar, double* grad, hipStream_t s) {
  GradArgs a{};
  a.n_env = n_env;
  a.offsets = offsets;
  a.pos = pos;
  a.Abar = Abar;
  a.grad = grad;
  a.onep_index = g->d_onep_index;
  a.ycoef = g->d_ycoef;
  a.P1 = g->P1;
  a.n_max = g->h.spec.n_max;
  a.l_max = g->h.spec.l_max;
  a.r_cut = g->h.spec.r_cut;
  const size_t lds = (size_t)g->P1 * 16 + g->onep_index.size() * 2 + 16;
  if (lds > g->max_lds) return fail(ACE_ERR_UNSUPPORTED, "one-particle basis too large for the gradient kernel");
  hipLaunchKernelGGL(grad_kernel, dim3((unsigned)grid_for(n_env)), dim3(kGradThreads), lds, s, a);
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

ace_status common_eval_checks(const ace_graph* g, const double* coeffs, int64_t n_env, const void* workspace,
                              size_t ws_bytes, uint32_t flags, size_t* need) {
  ace_status st = need_device(g);
  if (st != ACE_OK) return st;
  if (n_env < 0) return fail(ACE_ERR_INVALID_ARG, "n_env must be >= 0");
  if (n_env > ((int64_t)1 << 30)) return fail(ACE_ERR_INVALID_ARG, "n_env too large");
  if (flags & ~(ACE_FLAG_NAIVE | ACE_FLAG_CHECK)) return fail(ACE_ERR_INVALID_ARG, "unknown flag bits");
  if (n_env == 0) return ACE_OK;
  if (!coeffs) return fail(ACE_ERR_INVALID_ARG, "coeffs is NULL");
  *need = plan_workspace(g, n_env, nullptr).bytes;
  if (!workspace) return fail(ACE_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < *need)
    return fail(ACE_ERR_INVALID_ARG, "workspace too small: need " + std::to_string(*need) + " bytes, got " +
                                         std::to_string(ws_bytes));
  return ACE_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// exported functions
// ---------------------------------------------------------------------------
extern "C" {

const char* ace_last_error(void) { return g_error.c_str(); }

const char* ace_version(void) { return "ace-dag-gfx950 0.1"; }

ace_status ace_graph_build(const ace_basis_spec* spec, ace_graph** out) {
  if (!spec || !out) return fail(ACE_ERR_INVALID_ARG, "spec and out must be non-NULL");
  *out = nullptr;
  ace_graph* g = nullptr;
  try {
    g = new ace_graph();
    BuildSpec bs;
    bs.group = spec->group;
    bs.nu_max = spec->nu_max;
    bs.degree_max = spec->degree_max;
    bs.n_max = spec->n_max;
    bs.l_max = spec->l_max;
    bs.algorithm = spec->algorithm;
    bs.alg_n = spec->alg_n;
    bs.r_cut = spec->r_cut;
    build_graph(bs, g->h);
    make_schedule(g);
    make_stats(g);
  } catch (const std::invalid_argument& e) {
    delete g;
    return fail(ACE_ERR_INVALID_ARG, e.what());
  } catch (const std::bad_alloc&) {
    delete g;
    return fail(ACE_ERR_OUT_OF_MEMORY, "host allocation failed during graph build");
  } catch (const std::exception& e) {
    delete g;
    return fail(ACE_ERR_INTERNAL, e.what());
  }
  if (!(spec->build_flags & ACE_BUILD_HOST_ONLY)) {
    ace_status st = upload(g);
    if (st != ACE_OK) {
      ace_graph_free(g);
      return st;
    }
  }
  *out = g;
  return ACE_OK;
}

void ace_graph_free(ace_graph* g) {
  if (!g) return;
  if (g->dmem) (void)hipFree(g->dmem);
  delete g;
}

ace_status ace_graph_info(const ace_graph* g, ace_graph_stats* stats) {
  if (!g || !stats) return fail(ACE_ERR_INVALID_ARG, "graph and stats must be non-NULL");
  *stats = g->stats;
  return ACE_OK;
}

ace_status ace_graph_export(const ace_graph* g, int32_t* onep, int32_t* node_tuple, int32_t* parents,
                            int64_t* k_to_node) {
  if (!g) return fail(ACE_ERR_INVALID_ARG, "graph is NULL");
  const HostGraph& h = g->h;
  if (onep)
    for (int i = 0; i < h.P1; ++i) {
      onep[3 * i] = h.on_n[i];
      onep[3 * i + 1] = h.on_l[i];
      onep[3 * i + 2] = h.on_m[i];
    }
  if (node_tuple) std::memcpy(node_tuple, h.node_flat.data(), h.node_flat.size() * 4);
  if (parents) std::memcpy(parents, h.par.data(), h.par.size() * 4);
  if (k_to_node) std::memcpy(k_to_node, h.k_to_node.data(), h.k_to_node.size() * 8);
  return ACE_OK;
}

ace_status ace_graph_export_k(const ace_graph* g, int32_t* k_tuples) {
  if (!g || !k_tuples) return fail(ACE_ERR_INVALID_ARG, "graph and k_tuples must be non-NULL");
  std::memcpy(k_tuples, g->h.k_flat.data(), g->h.k_flat.size() * 4);
  return ACE_OK;
}

ace_status ace_workspace_size(const ace_graph* g, int64_t n_env, int64_t n_nbr, uint32_t flags, size_t* bytes) {
  (void)n_nbr;
  (void)flags;
  if (!g || !bytes) return fail(ACE_ERR_INVALID_ARG, "graph and bytes must be non-NULL");
  if (n_env < 0) return fail(ACE_ERR_INVALID_ARG, "n_env must be >= 0");
  if (!g->on_device) return fail(ACE_ERR_INVALID_ARG, "graph was built with ACE_BUILD_HOST_ONLY");
  *bytes = plan_workspace(g, n_env, nullptr).bytes;
  return ACE_OK;
}

ace_status ace_basis(const ace_graph* g, int64_t n_env, const int32_t* offsets, const double* pos, double* A,
                     void* stream) {
  ace_status st = need_device(g);
  if (st != ACE_OK) return st;
  if (n_env < 0) return fail(ACE_ERR_INVALID_ARG, "n_env must be >= 0");
  if (n_env == 0) return ACE_OK;
  if (!offsets || !pos || !A) return fail(ACE_ERR_INVALID_ARG, "offsets, pos and A must be non-NULL");
  return launch_basis(g, n_env, offsets, pos, reinterpret_cast<double2*>(A), (hipStream_t)stream);
}

ace_status ace_contract(const ace_graph* g, const double* coeffs, int64_t n_env, const double* A, double* phi,
                        double* Abar, void* workspace, size_t ws_bytes, uint32_t flags, void* stream) {
  size_t need = 0;
  ace_status st = common_eval_checks(g, coeffs, n_env, workspace, ws_bytes, flags, &need);
  if (st != ACE_OK || n_env == 0) return st;
  if (!A || !phi) return fail(ACE_ERR_INVALID_ARG, "A and phi must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  const Workspace w = plan_workspace(g, n_env, static_cast<char*>(workspace));
  if (flags & ACE_FLAG_NAIVE)
    return launch_naive(g, coeffs, n_env, reinterpret_cast<const double2*>(A), reinterpret_cast<double2*>(phi),
                        reinterpret_cast<double2*>(Abar), s);
  return launch_dag(g, coeffs, n_env, reinterpret_cast<const double2*>(A), reinterpret_cast<double2*>(phi),
                    reinterpret_cast<double2*>(Abar), w, s);
}

ace_status ace_eval(const ace_graph* g, const double* coeffs, int64_t n_env, const int32_t* offsets,
                    const double* pos, double* phi, void* workspace, size_t ws_bytes, uint32_t flags, void* stream) {
  size_t need = 0;
  ace_status st = common_eval_checks(g, coeffs, n_env, workspace, ws_bytes, flags, &need);
  if (st != ACE_OK || n_env == 0) return st;
  if (!offsets || !pos || !phi) return fail(ACE_ERR_INVALID_ARG, "offsets, pos and phi must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  if (flags & ACE_FLAG_CHECK) {
    st = check_offsets(offsets, n_env, -1, s);
    if (st != ACE_OK) return st;
  }
  const Workspace w = plan_workspace(g, n_env, static_cast<char*>(workspace));
  st = launch_basis(g, n_env, offsets, pos, w.A, s);
  if (st != ACE_OK) return st;
  if (flags & ACE_FLAG_NAIVE) return launch_naive(g, coeffs, n_env, w.A, reinterpret_cast<double2*>(phi), nullptr, s);
  return launch_dag(g, coeffs, n_env, w.A, reinterpret_cast<double2*>(phi), nullptr, w, s);
}

ace_status ace_eval_grad(const ace_graph* g, const double* coeffs, int64_t n_env, const int32_t* offsets,
                         const double* pos, double* phi, double* grad, void* workspace, size_t ws_bytes,
                         uint32_t flags, void* stream) {
  size_t need = 0;
  ace_status st = common_eval_checks(g, coeffs, n_env, workspace, ws_bytes, flags, &need);
  if (st != ACE_OK || n_env == 0) return st;
  if (!offsets || !pos || !phi || !grad)
    return fail(ACE_ERR_INVALID_ARG, "offsets, pos, phi and grad must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  if (flags & ACE_FLAG_CHECK) {
    st = check_offsets(offsets, n_env, -1, s);
    if (st != ACE_OK) return st;
  }
  const Workspace w = plan_workspace(g, n_env, static_cast<char*>(workspace));
  st = launch_basis(g, n_env, offsets, pos, w.A, s);
  if (st != ACE_OK) return st;
  if (flags & ACE_FLAG_NAIVE)
    st = launch_naive(g, coeffs, n_env, w.A, reinterpret_cast<double2*>(phi), w.Abar, s);
  else
    st = launch_dag(g, coeffs, n_env, w.A, reinterpret_cast<double2*>(phi), w.Abar, w, s);
  if (st != ACE_OK) return st;
  return launch_grad(g, n_env, offsets, pos, w.Abar, grad, s);
}

}  // extern "C"
