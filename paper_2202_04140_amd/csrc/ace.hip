// C ABI of the evaluator (declared in include/ace.h): graph build and
// upload, workspace sizing, and the launch sequences of ace_basis,
// ace_contract, ace_eval and ace_eval_grad.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cstdint>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
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
constexpr int kForestThreads = 512;
constexpr int kNaiveChunk = 16;     // naive kernel: consecutive tuples per lane and slice
constexpr int kBasisThreads = 256;
constexpr int kGradThreads = 256;   // planar gradient kernel
constexpr int kGradWave = 64;       // O(3) gradient kernel: one wave per block
constexpr int kArenaBlocks = 1024;
constexpr int kRematMaxSlots = 4096;   // remat factor fields are 16-bit LDS byte offsets
constexpr int64_t kRematMaxEntries = 1 << 26;   // coefficients plus entry positions of one remat schedule
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace
}  // namespace ace

// Workspace of ace_eval_grad_noalloc: a fixed device array, one copy on each
// device the library runs on, held until the process ends.  In host code its
// name is a stand-in, not a device address; host code uses only the address
// hipGetSymbolAddress returns for the current device (scratch_address below).
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

using namespace ace;

// ---------------------------------------------------------------------------
// graph object
// ---------------------------------------------------------------------------
// Tunable parameters of the forest schedule (ace_schedule_opts).
struct ScheduleOpts {
  int row_chunk = 32;      // resident-pair entries per row item at most
  int tree_chunk = 16;     // regular children per tree item at most
  int hot_columns = 4;     // hot-sibling register columns (0..4)
  int bank_schedule = 1;   // order lanes and columns by LDS bank group
  int block_threads = 512; // remat kernel block size; the forest kernel takes at most 512
  int schedule = 0;        // ACE_SCHEDULE_*
  int term_chunk = 64;     // remat: terms per lane item at most
  int pair_slots = -1;     // remat: precomputed one-particle pair products at most (-1: fill LDS)
  int env_per_block = 1;   // forest and remat: environments per block (1 or 2)
};

struct ace_graph {
  HostGraph h;
  ScheduleOpts opts;
  ace_graph_stats stats{};
  bool on_device = false;
  int device = -1;
  // evaluation schedule (host copies)
  int P1 = 0, S = 0, T = 0, slots = 0, depth = 0;
  int st_off[kMaxLayers + 2] = {0};
  int cl_off[kMaxLayers + 2] = {0};
  std::vector<int2> st_ab, cl_ab;
  std::vector<int32_t> st_k, cl_k, leaf_k;
  // naive schedule (naive_kernel): slices, factor indices, K index of every
  // coefficient position (-1: padding)
  std::vector<int4> nv_slice;
  std::vector<int16_t> nv_idx;
  std::vector<int32_t> nv_kmap;
  std::vector<OnepInfo> onep;
  std::vector<int16_t> onep_index;
  std::vector<int16_t> basis_prim;   // O(3): the functions with m >= 0
  std::vector<int32_t> gsrc;
  int grad_nb = 0;                 // gradient kernel: Abar entries per (l, m), padded to odd
  std::vector<double> ycoef;
  // device copies (one allocation)
  void* dmem = nullptr;
  int2 *d_st_ab = nullptr, *d_cl_ab = nullptr;
  int32_t *d_st_k = nullptr, *d_cl_k = nullptr, *d_leaf_k = nullptr;
  int4* d_nv_slice = nullptr;
  int32_t* d_nv_kmap = nullptr;
  int16_t *d_nv_idx = nullptr, *d_onep_index = nullptr, *d_basis_prim = nullptr;
  int32_t* d_gsrc = nullptr;
  OnepInfo* d_onep = nullptr;
  double* d_ycoef = nullptr;
  // LDS plan
  size_t max_lds = 0;
  bool fwd_xl = false;    // forward-only: value arena in LDS
  bool grad_xl = false;   // forward+reverse: value arena in LDS
  bool grad_al = false;   // forward+reverse: adjoint arena in LDS
  // forest schedule (forest_kernel): [0] over every tuple of K, [1] over one
  // tuple of each conjugate pair (coefficients as (Re, Im) weights)
  struct Forest {
    bool ok = false;
    bool fold = false;
    std::string why;
    int N2 = 0, nslot = 0, n_mslices = 0, n_tslices = 0;
    bool has_gc = false;
    std::vector<uint32_t> nu2_ab, it_ab;
    std::vector<int4> mr_slice, tr_slice;
    std::vector<uint16_t> mr_row, me_col, ch_s, gc_s;
    std::vector<int2> ch_g;
    std::vector<int32_t> kmap;
    std::vector<int32_t> kbar;       // folded: conjugate partner of each kmap entry (-1: self)
    int cs_leaf = 0, cs_nu2 = 0, cs_me = 0, cs_it = 0, cs_ch = 0, cs_gc = 0;
    uint32_t *d_nu2_ab = nullptr, *d_it_ab = nullptr;
    int4 *d_mr_slice = nullptr, *d_tr_slice = nullptr;
    uint16_t *d_mr_row = nullptr, *d_me_col = nullptr, *d_ch_s = nullptr, *d_gc_s = nullptr;
    int2* d_ch_g = nullptr;
    int32_t *d_kmap = nullptr, *d_kbar = nullptr;
    bool fwd_lds = false, grad_lds = false;
    bool full = false;               // full-adjoint mode fits in LDS
    int hot_slot[4] = {0, 0, 0, 0};  // most frequent childless-child siblings
    int n_items = 0;                 // tree items incl. slice padding (= 64 * n_tslices)
    int mr_wave[kMaxForestWaves + 1] = {0};   // wave w takes pair-row slices [mr_wave[w], mr_wave[w + 1])
    int tr_wave[kMaxForestWaves + 1] = {0};   // and tree slices [tr_wave[w], tr_wave[w + 1])
    int cs_hot = 0;                  // coefficients of the hot columns, [4][n_items]
    // full-adjoint mode: order-2 -> one-particle forwarding lists, cut into
    // chunks {one-particle slot, first entry, end entry, 0} of exactly
    // kForwardChunk entries (chunk c holds entries [c * kForwardChunk, ...),
    // padded with the zero slot)
    std::vector<int4> fw_ck;
    std::vector<uint32_t> fw_ent;
    int4* d_fw_ck = nullptr;
    uint32_t* d_fw_ent = nullptr;
  } fo[2];
  void* fmem = nullptr;
  // rematerialising schedule (remat_kernel): [0] forward only (each term in
  // one row), [1] with adjoint (each term in the rows of both parents),
  // [2], [3] the same over one tuple of each conjugate pair
  bool remat_ok = false;
  std::string remat_why;
  struct Remat {
    bool fold = false;             // conjugate pairs folded (coefficients as (Re, Im) weights)
    int nslices = 0, nitems = 0, cs_leaf = 0, cs_ent = 0;
    int hot[4] = {0, 0, 0, 0};
    std::vector<int4> slice;
    std::vector<uint64_t> rlo, rhi, olo, ohi;
    std::vector<int32_t> kmap;
    std::vector<uint32_t> pairs;   // pair products: one-particle slots a | b << 16
    std::vector<int32_t> kbar;     // folded: conjugate partner of each kmap entry (-1: self)
    int4* d_slice = nullptr;
    uint64_t *d_rlo = nullptr, *d_rhi = nullptr, *d_olo = nullptr, *d_ohi = nullptr;
    int32_t* d_kmap = nullptr;
    int32_t* d_kbar = nullptr;
    uint32_t* d_pairs = nullptr;
  } rm[4];   // forward only, with adjoint; the same two with conjugate pairs folded
  void* rmem = nullptr;
  bool remat_lds = false;          // the one-particle values and adjoints fit in LDS
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

// largest n and |m| of a planar basis (torus: n = 0, |m| <= D)
int planar_n(const HostGraph& h) { return h.spec.group == 2 ? std::min(h.spec.n_max, h.spec.degree_max) : 0; }
int planar_m(const HostGraph& h) {
  return h.spec.group == 2 ? std::min(h.spec.l_max, h.spec.degree_max) : h.spec.degree_max;
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

  // naive schedule: K is ordered by length, so the tuples of one length are
  // contiguous; each length is cut into slices of 64 lanes x kNaiveChunk
  // consecutive tuples per lane, padded with the constant-one slot P1
  if (P1 > 32766) throw std::length_error("too many one-particle functions for int16 tuples");
  g->nv_slice.clear();
  g->nv_idx.clear();
  g->nv_kmap.clear();
  for (int64_t b = 0; b < h.nK;) {
    const int nu = h.k_len[b];
    int64_t e = b;
    while (e < h.nK && h.k_len[e] == nu) ++e;
    const int64_t per_slice = 64LL * kNaiveChunk;
    for (int64_t s0 = b; s0 < e; s0 += per_slice) {
      if ((int64_t)g->nv_idx.size() + per_slice * nu > INT32_MAX)
        throw std::length_error("naive schedule larger than 2^31 entries");
      g->nv_slice.push_back(make_int4((int)g->nv_idx.size(), (int)g->nv_kmap.size(), nu, kNaiveChunk));
      for (int j = 0; j < kNaiveChunk; ++j) {
        for (int t = 0; t < nu; ++t)
          for (int lane = 0; lane < 64; ++lane) {
            const int64_t q = s0 + (int64_t)lane * kNaiveChunk + j;
            g->nv_idx.push_back(q < e ? (int16_t)h.k_flat[(size_t)q * h.width + t] : (int16_t)P1);
          }
      }
      for (int j = 0; j < kNaiveChunk; ++j)
        for (int lane = 0; lane < 64; ++lane) {
          const int64_t q = s0 + (int64_t)lane * kNaiveChunk + j;
          g->nv_kmap.push_back(q < e ? (int32_t)q : -1);
        }
    }
    b = e;
  }

  // one-particle tables (O(3) only)
  g->onep.clear();
  g->onep_index.clear();
  g->basis_prim.clear();
  g->gsrc.clear();
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
      o.l = (int8_t)l;
      o.am = (int8_t)am;
      o.k = (int8_t)h.on_k[i];
      o.neg = -1;
      g->onep.push_back(o);
      if (h.on_k[i] == 0) g->onep_index[(size_t)(n * (L + 1) + l) * W + (m + L)] = (int16_t)i;
    }
    // the basis kernel sums the m >= 0 functions only; an m > 0 function also
    // writes its -m partner (same n, l, k), a sign-flipped copy of its sums
    std::map<std::array<int, 4>, int> where;
    for (int i = 0; i < P1; ++i) where[{h.on_n[i], h.on_l[i], h.on_m[i], h.on_k[i]}] = i;
    for (int i = 0; i < P1; ++i) {
      if (h.on_m[i] < 0) continue;
      g->basis_prim.push_back((int16_t)i);
      if (h.on_m[i] > 0) {
        const auto it = where.find({h.on_n[i], h.on_l[i], -h.on_m[i], h.on_k[i]});
        if (it == where.end()) throw std::runtime_error("one-particle set without the -m partner of a function");
        g->onep[i].neg = (int16_t)it->second;
      }
    }
    make_ycoef(L, g->ycoef);
    // the gradient kernel's staged adjoint: position (l (l + 1) / 2 + m) NB +
    // n K1 + k, m >= 0, combines the functions (n, l, +-m, k); its pair of
    // sources is (index of +m or -1, index of -m encoded as i for even m and
    // -2 - i for odd m, or -1: absent or m = 0).  The block of one (l, m) is
    // padded to an odd length NB, so that lanes reading different (l, m)
    // spread over the LDS bank groups.
    const int K1 = h.spec.k_max + 1;
    const int NY = (L + 1) * (L + 2) / 2;
    g->grad_nb = ((N + 1) * K1) | 1;
    g->gsrc.assign((size_t)NY * g->grad_nb * 2, -1);
    for (int i = 0; i < P1; ++i) {
      const int l = h.on_l[i], m = h.on_m[i], am = m < 0 ? -m : m;
      const size_t slot = (size_t)((l * (l + 1)) / 2 + am) * g->grad_nb + h.on_n[i] * K1 + h.on_k[i];
      if (m >= 0)
        g->gsrc[2 * slot] = i;
      else
        g->gsrc[2 * slot + 1] = (am & 1) ? -2 - i : i;
    }
  } else {
    // planar groups: phi = R_n (Re E, sim Im E), E = u^{|m|}, sim = s sign(m) with
    // s = +1 (torus, e^{+i m theta}) or -1 (SO(2), e^{-i m theta}); onep_index
    // holds the planar (n, m) -> i table [(N+1)][(2M+1)]
    const int N = planar_n(h), M = planar_m(h), W = 2 * M + 1;
    const int s = h.spec.group == 1 ? 1 : -1;
    g->onep_index.assign((size_t)(N + 1) * W, (int16_t)-1);
    for (int i = 0; i < P1; ++i) {
      const int n = h.on_n[i], m = h.on_m[i];
      OnepInfo o{};
      o.n = (int16_t)n;
      o.am = (int8_t)(m < 0 ? -m : m);
      o.yoff = o.am;
      o.sre = 1;
      o.sim = (int8_t)(m == 0 ? 1 : (m > 0 ? s : -s));
      o.l = o.am;
      o.neg = -1;
      g->onep.push_back(o);
      g->onep_index[(size_t)n * W + (m + M)] = (int16_t)i;
    }
  }
}

// ---------------------------------------------------------------------------
// Forest schedule (see forest_kernel in kernels.hip).
// ---------------------------------------------------------------------------


// ---------------------------------------------------------------------------
// LDS bank scheduling.  A 16-byte LDS gather of one wave is served in four
// quarters of 16 lanes; a quarter costs as many cycles as the largest number
// of its lanes whose slots share a bank group (slot mod 16).  Entries of a
// lane may be taken in any order, so each column is chosen by a bipartite
// matching of the quarter's lanes to bank groups.
// ---------------------------------------------------------------------------
struct Ent {
  int32_t slot;  // resident slot read at this position
  int32_t pay;   // caller's payload; -1 marks padding (coefficient 0)
};

bool kuhn(int l, const std::vector<uint32_t>& avail, const int* border, std::vector<int>& bank_of,
          std::vector<int>& lane_of, uint32_t& seen) {
  for (int bi = 0; bi < 16; ++bi) {
    const int b = border[bi];
    if (!(avail[l] & (1u << b)) || (seen & (1u << b))) continue;
    seen |= 1u << b;
    if (lane_of[b] < 0 || kuhn(lane_of[b], avail, border, bank_of, lane_of, seen)) {
      lane_of[b] = l;
      bank_of[l] = b;
      return true;
    }
  }
  return false;
}

// lanes[l]: entries of lane l (l < 64), consumed.  Returns ncol columns of 64
// positions.  Padding reads slot pad_slot(bank) with a bank still free.
template <typename PadSlot>
std::vector<std::vector<Ent>> bank_columns(std::vector<std::vector<Ent>>& lanes, int ncol, PadSlot pad_slot) {
  std::vector<std::vector<Ent>> out(ncol, std::vector<Ent>(64, Ent{-1, -1}));
  lanes.resize(64);
  for (int j = 0; j < ncol; ++j)
    for (int q = 0; q < 4; ++q) {
      std::vector<uint32_t> avail(16, 0);
      int demand[16] = {0};
      for (int i = 0; i < 16; ++i)
        for (const Ent& e : lanes[16 * q + i]) {
          avail[i] |= 1u << (e.slot & 15);
          demand[e.slot & 15] += 1;
        }
      // banks with the most remaining entries first; lanes with the least slack first
      int border[16];
      for (int b = 0; b < 16; ++b) border[b] = b;
      std::stable_sort(border, border + 16, [&](int x, int y) { return demand[x] > demand[y]; });
      int lorder[16];
      for (int i = 0; i < 16; ++i) lorder[i] = i;
      std::stable_sort(lorder, lorder + 16,
                       [&](int x, int y) { return lanes[16 * q + x].size() > lanes[16 * q + y].size(); });
      std::vector<int> bank_of(16, -1), lane_of(16, -1);
      for (int ii = 0; ii < 16; ++ii) {
        const int i = lorder[ii];
        uint32_t seen = 0;
        if (avail[i]) kuhn(i, avail, border, bank_of, lane_of, seen);
      }
      uint32_t used = 0;
      std::vector<int> pend;
      for (int i = 0; i < 16; ++i) {
        std::vector<Ent>& L = lanes[16 * q + i];
        const int left = ncol - j;
        if (bank_of[i] >= 0) {
          auto it = std::find_if(L.begin(), L.end(), [&](const Ent& e) { return (e.slot & 15) == bank_of[i]; });
          out[j][16 * q + i] = *it;
          L.erase(it);
          used |= 1u << bank_of[i];
        } else if (!L.empty() && (int)L.size() >= left) {
          out[j][16 * q + i] = L.front();   // no slack left: take it despite the conflict
          used |= 1u << (L.front().slot & 15);
          L.erase(L.begin());
        } else {
          pend.push_back(i);                // padding now (the lane has slack)
        }
      }
      for (int i : pend) {
        int b = 0;
        while (b < 15 && (used & (1u << b))) ++b;
        used |= 1u << b;
        out[j][16 * q + i] = Ent{pad_slot(b), -1};
      }
    }
  return out;
}

// Permutation of up to 64 items into lanes: each goes to a quarter in which
// its key banks are not yet used, if any has room.
std::vector<int> bank_lanes(const std::vector<std::pair<int, int>>& keys) {
  std::vector<int> lane(keys.size(), -1);
  uint32_t ua[4] = {0, 0, 0, 0}, ub[4] = {0, 0, 0, 0};
  int fill[4] = {0, 0, 0, 0};
  for (size_t i = 0; i < keys.size(); ++i) {
    const uint32_t ma = 1u << (keys[i].first & 15), mb = keys[i].second < 0 ? 0u : 1u << (keys[i].second & 15);
    int best = -1, bestc = 99;
    for (int q = 0; q < 4; ++q) {
      if (fill[q] >= 16) continue;
      const int c = ((ua[q] & ma) ? 1 : 0) + ((ub[q] & mb) ? 1 : 0);
      if (c < bestc) {
        bestc = c;
        best = q;
      }
    }
    lane[i] = 16 * best + fill[best]++;
    ua[best] |= ma;
    ub[best] |= mb;
  }
  return lane;
}

// In-order alternatives (no bank scheduling).
std::vector<std::vector<Ent>> plain_columns(std::vector<std::vector<Ent>>& lanes, int ncol, int zero) {
  std::vector<std::vector<Ent>> out(ncol, std::vector<Ent>(64, Ent{zero, -1}));
  for (int l = 0; l < (int)lanes.size() && l < 64; ++l)
    for (int j = 0; j < (int)lanes[l].size(); ++j) out[j][l] = lanes[l][j];
  return out;
}

std::vector<int> plain_lanes(int n) {
  std::vector<int> v(n);
  for (int i = 0; i < n; ++i) v[i] = i;
  return v;
}

std::vector<int64_t> conj_partners(const HostGraph& h);

// which = 0: every tuple of K carries its coefficient.  which = 1 (folded):
// only the tuple of smaller index of each conjugate pair does, with the
// partner recorded beside its coefficient position; the other tuple stays
// in the schedule only as a parent, with coefficient 0.
void make_forest(ace_graph* g, int which) {
  const HostGraph& h = g->h;
  const int64_t V = h.n_nodes();
  const int P1 = h.P1;
  ace_graph::Forest& F = g->fo[which];
  F = ace_graph::Forest{};
  F.fold = which == 1;
  auto fail_forest = [&](const char* why) { F.why = why; };
  std::vector<int64_t> kbar;
  if (F.fold) {
    try {
      kbar = conj_partners(h);
    } catch (const std::logic_error& e) {
      return fail_forest("no conjugate pairs");
    }
  }
  // tuple of K whose coefficient node v carries, or -1
  std::vector<int32_t> nk(V, -1);
  for (int64_t v = 0; v < V; ++v) {
    const int32_t q = h.node_k[v];
    nk[v] = q >= 0 && (!F.fold || kbar[q] >= q) ? q : -1;
  }
  // liveness and live children (parents precede children in insertion order)
  std::vector<uint8_t> live(V, 0);
  for (int64_t v = 0; v < V; ++v) live[v] = nk[v] >= 0;
  std::vector<int32_t> nlc(V, 0);
  for (int64_t v = V - 1; v >= P1; --v) {
    if (!live[v]) continue;
    const int32_t a = h.par[2 * v], b = h.par[2 * v + 1];
    live[a] = live[b] = 1;
    nlc[a] += 1;
    nlc[b] += 1;
  }
  // resident slots: one-particle nodes, ZERO = P1, live order-2 nodes
  std::vector<int32_t> slot(V, -1);
  for (int i = 0; i < P1; ++i) slot[i] = i;
  std::vector<int32_t> nu2;
  for (int64_t v = P1; v < V; ++v)
    if (live[v] && h.layer[v] == 1) {
      slot[v] = P1 + 1 + (int32_t)nu2.size();
      nu2.push_back((int32_t)v);
    }
  const int nslot = P1 + 1 + (int)nu2.size();
  if (nslot > 65535) return fail_forest("more than 65535 resident slots");
  // classify product nodes above order 2
  std::vector<int32_t> primary(V, -1), sib(V, -1);
  std::vector<int32_t> roots, pairs;
  for (int64_t v = P1; v < V; ++v) {
    if (!live[v] || h.layer[v] < 2) continue;
    const int32_t a = h.par[2 * v], b = h.par[2 * v + 1];
    const bool ra = slot[a] >= 0, rb = slot[b] >= 0;
    if (ra && rb) {
      (nlc[v] > 0 ? roots : pairs).push_back((int32_t)v);
    } else if (ra || rb) {
      primary[v] = ra ? b : a;
      sib[v] = slot[ra ? a : b];
    } else {
      return fail_forest("a node with two non-resident parents");
    }
  }
  std::vector<std::vector<int32_t>> kids(V);
  for (int64_t v = P1; v < V; ++v)
    if (primary[v] >= 0) kids[primary[v]].push_back((int32_t)v);
  for (int64_t v = P1; v < V; ++v)
    if (live[v] && h.layer[v] >= 2 && (int64_t)kids[v].size() != nlc[v])
      return fail_forest("inconsistent child lists");
  bool has_gc = false;
  for (int32_t r : roots)
    for (int32_t c : kids[r])
      if (!kids[c].empty()) {
        has_gc = true;
        for (int32_t gch : kids[c])
          if (!kids[gch].empty()) return fail_forest("trees deeper than two levels");
      }
  F.has_gc = has_gc;
  F.N2 = (int)nu2.size();
  F.nslot = nslot;

  // ---- hot siblings: the most frequent siblings of childless tree children get
  // a fixed column per item, accumulated in registers (no atomics per child) ----
  {
    std::vector<int64_t> freq(nslot, 0);
    for (int32_t r : roots)
      for (int32_t c : kids[r])
        if (kids[c].empty()) freq[sib[c]] += 1;
    std::vector<int32_t> order(nslot);
    for (int i = 0; i < nslot; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return freq[x] > freq[y]; });
    for (int h = 0; h < 4; ++h) {
      const int sl = order[h];
      F.hot_slot[h] = (h < g->opts.hot_columns && sl != P1 && freq[sl] * 16 >= (int64_t)roots.size() &&
                        freq[sl] > 0) ? sl : P1;
    }
  }
  auto hot_col = [&](int slot_) {
    for (int h = 0; h < 4; ++h)
      if (F.hot_slot[h] != P1 && F.hot_slot[h] == slot_) return h;
    return -1;
  };
  // ---- tree items: root + hot columns + a chunk of at most kTreeChunk other children ----
  struct Item {
    int32_t root, c0, c1, ngc;
    int32_t hot[4];  // child node in each hot column, or -1
  };
  std::vector<Item> items;
  for (int32_t r : roots) {
    std::vector<int32_t> reg;
    int32_t hot[4] = {-1, -1, -1, -1};
    for (int32_t c : kids[r]) {
      const int hc = kids[c].empty() ? hot_col(sib[c]) : -1;
      if (hc >= 0 && hot[hc] < 0)
        hot[hc] = c;
      else
        reg.push_back(c);
    }
    kids[r] = reg;  // the regular children, in order
    const int n = (int)reg.size();
    int c0 = 0;
    do {
      const int c1 = std::min(n, c0 + g->opts.tree_chunk);
      int ngc = 0;
      for (int j = c0; j < c1; ++j) ngc += (int)kids[reg[j]].size();
      Item it{r, c0, c1, ngc, {-1, -1, -1, -1}};
      if (c0 == 0)
        for (int h = 0; h < 4; ++h) it.hot[h] = hot[h];
      items.push_back(it);
      c0 = c1;
    } while (c0 < n);
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) {
    if (x.c1 - x.c0 != y.c1 - y.c0) return x.c1 - x.c0 > y.c1 - y.c0;
    return x.ngc > y.ngc;
  });
  const uint32_t zz = (uint32_t)P1 | ((uint32_t)P1 << 16);
  // Pack items into slices of 64 lanes.  Items arrive sorted by size; each
  // goes to the first slice of a small window of open slices in which no
  // other lane pushes to the same root parents (same-address LDS atomics in
  // one instruction serialise), else to the first slice with room.
  std::vector<std::vector<int>> slices;
  {
    // per size class (items with the same regular-child count, which keeps
    // slices free of column padding): the minimal number of slices, each item
    // to the slice with room whose lanes share the fewest root parents with it
    int i0 = 0;
    while (i0 < (int)items.size()) {
      int i1 = i0;
      while (i1 < (int)items.size() && items[i1].c1 - items[i1].c0 == items[i0].c1 - items[i0].c0) ++i1;
      const int S = (i1 - i0 + 63) / 64;
      const int first = (int)slices.size();
      slices.resize(first + S);
      std::vector<std::vector<int32_t>> ta(S), tb(S);
      for (int i = i0; i < i1; ++i) {
        const int32_t a = slot[h.par[2 * items[i].root]], b = slot[h.par[2 * items[i].root + 1]];
        int best = -1, bestc = 1 << 30;
        for (int q = 0; q < S; ++q) {
          if (slices[first + q].size() >= 64) continue;
          const int c = (int)std::count(ta[q].begin(), ta[q].end(), a) + (int)std::count(tb[q].begin(), tb[q].end(), b);
          if (c < bestc) {
            bestc = c;
            best = q;
          }
        }
        slices[first + best].push_back(i);
        ta[best].push_back(a);
        tb[best].push_back(b);
      }
      i0 = i1;
    }
  }
  const int nts = (int)slices.size();
  std::vector<int32_t> k_it((size_t)nts * 64, -1), k_ch, k_gc;
  std::vector<int32_t> item_pos(items.size(), -1);   // item -> lane index sl*64 + l
  F.it_ab.assign((size_t)nts * 64, zz);
  F.tr_slice.assign(nts, make_int4(0, 0, 0, 0));
  F.ch_s.clear();
  F.ch_g.clear();
  F.gc_s.clear();
  // a slot in a given bank group for padding (one-particle slots 0..15)
  auto pad_slot = [&](int bank) { return P1 > 15 ? bank : P1; };
  for (int sl = 0; sl < nts; ++sl) {
    const int nl = (int)slices[sl].size();
    // lanes: root parents spread over bank groups per quarter
    std::vector<std::pair<int, int>> keys(nl);
    for (int l = 0; l < nl; ++l) {
      const Item& it = items[slices[sl][l]];
      keys[l] = {slot[h.par[2 * it.root]], slot[h.par[2 * it.root + 1]]};
    }
    const std::vector<int> lane_of_item = g->opts.bank_schedule ? bank_lanes(keys) : plain_lanes(nl);
    // children: any order within an item; bank-matched per column
    std::vector<std::vector<Ent>> lanes(64);
    int ncol = 0;
    for (int l = 0; l < nl; ++l) {
      const Item& it = items[slices[sl][l]];
      for (int j = it.c0; j < it.c1; ++j) lanes[lane_of_item[l]].push_back(Ent{sib[kids[it.root][j]], kids[it.root][j]});
      ncol = std::max(ncol, it.c1 - it.c0);
    }
    const std::vector<std::vector<Ent>> cols =
        g->opts.bank_schedule ? bank_columns(lanes, ncol, pad_slot) : plain_columns(lanes, ncol, P1);
    const int nmax = ncol;
    const int base = (int)F.ch_s.size();
    F.tr_slice[sl] = make_int4(sl * 64, base, nmax, 0);
    F.ch_s.resize(base + (size_t)nmax * 64, (uint16_t)P1);
    F.ch_g.resize(base + (size_t)nmax * 64, make_int2(0, 0));
    k_ch.resize(base + (size_t)nmax * 64, -1);
    for (int l = 0; l < nl; ++l) {
      const Item& it = items[slices[sl][l]];
      const int idx = sl * 64 + lane_of_item[l];
      item_pos[slices[sl][l]] = idx;
      const int32_t a = h.par[2 * it.root], b = h.par[2 * it.root + 1];
      F.it_ab[idx] = (uint32_t)slot[a] | ((uint32_t)slot[b] << 16);
      k_it[idx] = it.c0 == 0 ? nk[it.root] : -1;
    }
    for (int j = 0; j < nmax; ++j)
      for (int l = 0; l < 64; ++l) {
        const Ent& en = cols[j][l];
        const int pos = base + j * 64 + l;
        F.ch_s[pos] = (uint16_t)en.slot;
        if (en.pay < 0) continue;   // padding: coefficient 0
        const int32_t c = en.pay;
        k_ch[pos] = nk[c];
        if (!kids[c].empty()) {
          const int gb = (int)F.gc_s.size();
          for (int32_t gch : kids[c]) {
            F.gc_s.push_back((uint16_t)sib[gch]);
            k_gc.push_back(nk[gch]);
          }
          F.ch_g[pos] = make_int2(gb, (int)F.gc_s.size());
        } else if (nk[c] < 0) {
          return fail_forest("childless auxiliary child");
        }
      }
  }
  F.n_tslices = nts;
  F.n_items = nts * 64;
  std::vector<int32_t> k_hot((size_t)4 * nts * 64, -1);
  for (size_t i = 0; i < items.size(); ++i)
    for (int hc = 0; hc < 4; ++hc)
      if (items[i].hot[hc] >= 0) k_hot[(size_t)hc * nts * 64 + item_pos[i]] = nk[items[i].hot[hc]];

  // ---- resident-pair rows ----
  std::vector<std::vector<std::pair<uint16_t, int32_t>>> rows(nslot);
  // an invariant order-2 node u = a * b contributes c_u x_a x_b: a pair of
  // one-particle slots, so it joins M instead of needing its own pushes
  for (int32_t u : nu2)
    if (nk[u] >= 0) pairs.push_back(u);
  for (int32_t w : pairs) {
    const int sa = slot[h.par[2 * w]], sb = slot[h.par[2 * w + 1]];
    const int32_t k = nk[w];
    if (k < 0) return fail_forest("childless auxiliary pair");
    if (sa == sb) {
      rows[sa].push_back({(uint16_t)sa, -2 - k});  // M_uu = 2 c
    } else {
      rows[sa].push_back({(uint16_t)sb, k});
      rows[sb].push_back({(uint16_t)sa, k});
    }
  }
  struct Row {
    int32_t row, e0, e1;
  };
  std::vector<Row> rch;
  for (int r = 0; r < nslot; ++r)
    for (int e0 = 0; e0 < (int)rows[r].size(); e0 += g->opts.row_chunk)
      rch.push_back({r, e0, std::min((int)rows[r].size(), e0 + g->opts.row_chunk)});
  std::stable_sort(rch.begin(), rch.end(), [](const Row& x, const Row& y) { return x.e1 - x.e0 > y.e1 - y.e0; });
  const int nms = (int)((rch.size() + 63) / 64);
  F.mr_slice.assign(nms, make_int4(0, 0, 0, 0));
  F.mr_row.assign((size_t)nms * 64, (uint16_t)P1);
  F.me_col.clear();
  std::vector<int32_t> k_me;
  for (int sl = 0; sl < nms; ++sl) {
    const int nl = std::min(64, (int)rch.size() - sl * 64);
    std::vector<std::pair<int, int>> keys(nl);
    int nmax = 0;
    for (int l = 0; l < nl; ++l) {
      keys[l] = {rch[sl * 64 + l].row, -1};
      nmax = std::max(nmax, rch[sl * 64 + l].e1 - rch[sl * 64 + l].e0);
    }
    const std::vector<int> lane_of_row = g->opts.bank_schedule ? bank_lanes(keys) : plain_lanes(nl);
    std::vector<std::vector<Ent>> lanes(64);
    for (int l = 0; l < nl; ++l) {
      const Row& rc = rch[sl * 64 + l];
      for (int j = rc.e0; j < rc.e1; ++j) lanes[lane_of_row[l]].push_back(Ent{rows[rc.row][j].first, rows[rc.row][j].second});
    }
    const std::vector<std::vector<Ent>> cols =
        g->opts.bank_schedule ? bank_columns(lanes, nmax, pad_slot) : plain_columns(lanes, nmax, P1);
    const int base = (int)F.me_col.size();
    F.mr_slice[sl] = make_int4(sl * 64, base, nmax, 0);
    F.me_col.resize(base + (size_t)nmax * 64, (uint16_t)P1);
    k_me.resize(base + (size_t)nmax * 64, -1);
    for (int l = 0; l < nl; ++l) F.mr_row[sl * 64 + lane_of_row[l]] = (uint16_t)rch[sl * 64 + l].row;
    for (int j = 0; j < nmax; ++j)
      for (int l = 0; l < 64; ++l) {
        const int pos = base + j * 64 + l;
        F.me_col[pos] = (uint16_t)cols[j][l].slot;
        k_me[pos] = cols[j][l].pay;   // padding: -1, coefficient 0
      }
  }
  F.n_mslices = nms;

  // ---- slices to waves: longest first to the least loaded wave (cost
  // estimates in units of one pair-row entry), then each wave's pair-row and
  // tree slices made contiguous, so that the block's waves finish together ----
  {
    const int nw = std::max(1, std::min(kMaxForestWaves, g->opts.block_threads / 64));
    struct SC {
      double cost;
      int tree, idx;
    };
    std::vector<SC> sc;
    for (int s = 0; s < nms; ++s) sc.push_back({1.0 + F.mr_slice[s].z, 0, s});
    for (int s = 0; s < nts; ++s) {
      const int4 d = F.tr_slice[s];
      int gcmax = 0;
      if (!F.gc_s.empty())
        for (int l = 0; l < 64; ++l) {
          int n = 0;
          for (int j = 0; j < d.z; ++j) {
            const int2 r = F.ch_g[d.y + j * 64 + l];
            n += r.y - r.x;
          }
          gcmax = std::max(gcmax, n);
        }
      sc.push_back({6.0 + 3.0 * d.z + 3.0 * gcmax, 1, s});
    }
    std::stable_sort(sc.begin(), sc.end(), [](const SC& a, const SC& b) { return a.cost > b.cost; });
    std::vector<double> load(nw, 0.0);
    std::vector<std::vector<int>> rows_of(nw), trees_of(nw);
    for (const SC& c : sc) {
      const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[w] += c.cost;
      (c.tree ? trees_of : rows_of)[w].push_back(c.idx);
    }
    std::vector<int4> mr(F.mr_slice), tr(F.tr_slice);
    int im = 0, it = 0;
    for (int w = 0; w < nw; ++w) {
      F.mr_wave[w] = im;
      F.tr_wave[w] = it;
      for (int s : rows_of[w]) F.mr_slice[im++] = mr[s];
      for (int s : trees_of[w]) F.tr_slice[it++] = tr[s];
    }
    for (int w = nw; w <= kMaxForestWaves; ++w) {
      F.mr_wave[w] = im;
      F.tr_wave[w] = it;
    }
  }

  // ---- order-2 nodes, one-particle coefficients, coefficient map ----
  F.nu2_ab.resize(nu2.size());
  std::vector<int32_t> k_nu2(nu2.size());
  for (size_t u = 0; u < nu2.size(); ++u) {
    const int32_t v = nu2[u];
    F.nu2_ab[u] = (uint32_t)slot[h.par[2 * v]] | ((uint32_t)slot[h.par[2 * v + 1]] << 16);
    if (slot[h.par[2 * v]] >= P1 || slot[h.par[2 * v + 1]] >= P1) return fail_forest("order-2 node without one-particle parents");
    k_nu2[u] = -1;  // carried by the resident-pair matrix
  }
  F.kmap.clear();
  auto put = [&](const std::vector<int32_t>& part) {
    const int off = (int)F.kmap.size();
    F.kmap.insert(F.kmap.end(), part.begin(), part.end());
    return off;
  };
  F.cs_it = put(k_it);
  F.cs_ch = put(k_ch);
  F.cs_gc = put(k_gc);
  F.cs_hot = put(k_hot);
  F.cs_me = put(k_me);
  F.cs_nu2 = put(k_nu2);
  std::vector<int32_t> k_leaf(nk.begin(), nk.begin() + P1);
  F.cs_leaf = put(k_leaf);
  if (F.fold) {
    F.kbar.assign(F.kmap.size(), -1);
    for (size_t i = 0; i < F.kmap.size(); ++i) {
      const int32_t k = F.kmap[i];
      if (k == -1) continue;
      const int64_t q = k >= 0 ? k : -2 - k;
      if (kbar[q] != q) F.kbar[i] = (int32_t)kbar[q];
    }
  }
  // forwarding lists: one-particle node i receives abar_u x_j from every
  // order-2 node u = i * j (a square u = i * i contributes twice)
  {
    std::vector<std::vector<uint32_t>> fl(P1);
    for (size_t u = 0; u < nu2.size(); ++u) {
      const uint32_t q = F.nu2_ab[u];
      const uint32_t a = q & 0xffffu, b = q >> 16;
      const uint32_t us = (uint32_t)(P1 + 1 + u);
      fl[a].push_back(us | (b << 16));
      fl[b].push_back(us | (a << 16));
    }
    // chunks of a fixed size, padded with the zero slot (whose value is 0):
    // a one-particle node that is a parent of many order-2 nodes would
    // otherwise hold one lane in a long serial loop, and a fixed size lets a
    // lane load all its entries at once.  Chunks go in rounds (the first
    // chunk of every node, then the second, ...), so that the lanes of a
    // wave add their sums to different nodes.
    F.fw_ck.clear();
    F.fw_ent.clear();
    const uint32_t pad = (uint32_t)P1 | ((uint32_t)P1 << 16);   // the zero slot, twice
    for (size_t r = 0;; ++r) {
      bool any = false;
      for (int i = 0; i < P1; ++i) {
        const size_t b0 = r * kForwardChunk;
        if (b0 >= fl[i].size()) continue;
        any = true;
        const int c = (int)F.fw_ent.size();
        for (size_t j = b0; j < b0 + kForwardChunk; ++j) F.fw_ent.push_back(j < fl[i].size() ? fl[i][j] : pad);
        F.fw_ck.push_back(make_int4(i, c, c + kForwardChunk, 0));
      }
      if (!any) break;
    }
  }
  if (F.kmap.size() > (size_t)(INT32_MAX / 16) || F.me_col.size() > (size_t)(INT32_MAX / 2) ||
      F.ch_s.size() > (size_t)(INT32_MAX / 2))
    return fail_forest("forest schedule larger than 2^27 coefficients");
  F.ok = true;
}

// Host emulation of forest_kernel for one environment, with the same
// indices, padding and forwarding, every index bounds-checked.  Used by the
// tests to validate a schedule without a GPU.  Every coefficient is a pair
// (Re weight, Im weight): (c, c) unfolded, (c_k + c_kbar, c_k - c_kbar)
// folded; Re phi takes the Re weights, Im phi the Im weights, the adjoint
// the Re weights.  Returns false on a bad index.
bool forest_emulate(const ace_graph* g, int which, const double* coeffs, const double* A, double* phi, double* Abar,
                    bool full) {
  using cd = std::complex<double>;
  const ace_graph::Forest& F = g->fo[which];
  const int P1 = g->P1, ZERO = P1;
  std::vector<double> cr(F.kmap.size(), 0.0), ci(F.kmap.size(), 0.0);
  for (size_t i = 0; i < cr.size(); ++i) {
    const int k = F.kmap[i];
    if (k >= g->h.nK || -2 - k >= g->h.nK) return false;
    if (k == -1) continue;
    const int q = k >= 0 ? k : -2 - k;
    const double sc = k >= 0 ? 1.0 : 2.0;
    const int kb = F.fold ? F.kbar.at(i) : -1;
    if (kb >= g->h.nK) return false;
    cr[i] = sc * (kb >= 0 ? coeffs[q] + coeffs[kb] : coeffs[q]);
    ci[i] = sc * (kb >= 0 ? coeffs[q] - coeffs[kb] : coeffs[q]);
  }
  std::vector<cd> x(F.nslot), ab(full ? F.nslot : P1 + 1, cd(0.0, 0.0));
  auto X = [&](int s) -> cd& {
    if (s < 0 || s >= F.nslot) throw std::out_of_range("slot");
    return x[s];
  };
  auto push = [&](int s, cd d) {
    if (full || s <= P1) {
      ab.at(s) += d;
    } else {
      const uint32_t q = F.nu2_ab.at(s - P1 - 1);
      const int a = (int)(q & 0xffffu), b = (int)(q >> 16);
      ab.at(a) += d * X(b);
      ab.at(b) += d * X(a);
    }
  };
  try {
    for (int i = 0; i < P1; ++i) {
      x[i] = cd(A[2 * i], A[2 * i + 1]);
      ab[i] = cd(cr.at(F.cs_leaf + i), 0.0);
    }
    x[ZERO] = 0.0;
    ab[ZERO] = 0.0;
    cd accr = 0.0, acci = 0.0;   // phi = Re accr + i Im acci
    for (int i = 0; i < P1; ++i) {
      accr += cr.at(F.cs_leaf + i) * x[i];
      acci += ci.at(F.cs_leaf + i) * x[i];
    }
    for (int u = 0; u < F.N2; ++u) {
      const uint32_t q = F.nu2_ab.at(u);
      const int a = (int)(q & 0xffffu), b = (int)(q >> 16);
      if (a >= P1 || b >= P1) return false;
      const cd xu = X(a) * X(b);
      X(P1 + 1 + u) = xu;
      // an invariant order-2 node's own term is a pair-matrix entry
      if (F.kmap.at(F.cs_nu2 + u) != -1) return false;
    }
    for (int s = 0; s < F.n_mslices; ++s) {
      const int4 sl = F.mr_slice.at(s);
      for (int lane = 0; lane < 64; ++lane) {
        const int row = F.mr_row.at(sl.x + lane);
        const cd xu = X(row);
        cd yr = 0.0, yi = 0.0;
        for (int j = 0; j < sl.z; ++j) {
          const int pos = sl.y + j * 64 + lane;
          yr += cr.at(F.cs_me + pos) * X(F.me_col.at(pos));
          yi += ci.at(F.cs_me + pos) * X(F.me_col.at(pos));
        }
        accr += 0.5 * xu * yr;
        acci += 0.5 * xu * yi;
        if (row != ZERO) push(row, yr);
      }
    }
    cd hacc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < F.n_tslices; ++s) {
      const int4 sl = F.tr_slice.at(s);
      for (int lane = 0; lane < 64; ++lane) {
        const int item = sl.x + lane;
        const uint32_t q = F.it_ab.at(item);
        const int a = (int)(q & 0xffffu), b = (int)(q >> 16);
        const cd xa = X(a), xb = X(b), xv = xa * xb;
        cd tr = cr.at(F.cs_it + item), ti = ci.at(F.cs_it + item), asum = 0.0;
        for (int hc = 0; hc < 4; ++hc) {
          const size_t hp = (size_t)F.cs_hot + (size_t)hc * F.n_items + item;
          tr += cr.at(hp) * X(F.hot_slot[hc]);
          ti += ci.at(hp) * X(F.hot_slot[hc]);
          hacc[hc] += cr.at(hp) * xv;
        }
        for (int j = 0; j < sl.z; ++j) {
          const int pos = sl.y + j * 64 + lane;
          const int sidx = F.ch_s.at(pos);
          const double c = cr.at(F.cs_ch + pos), c2 = ci.at(F.cs_ch + pos);
          const cd xs = X(sidx);
          const int2 gg = F.ch_g.at(pos);
          if (gg.x == gg.y) {
            tr += c * xs;
            ti += c2 * xs;
            if (c != 0.0) push(sidx, c * xv);
          } else {
            const cd xw = xv * xs;
            cd awr = c, awi = c2;
            for (int k = gg.x; k < gg.y; ++k) {
              const int sg = F.gc_s.at(k);
              awr += cr.at(F.cs_gc + k) * X(sg);
              awi += ci.at(F.cs_gc + k) * X(sg);
              push(sg, cr.at(F.cs_gc + k) * xw);
            }
            accr += xw * awr;
            acci += xw * awi;
            push(sidx, awr * xv);
            asum += awr * xs;
          }
        }
        accr += xv * tr;
        acci += xv * ti;
        if (q != ((uint32_t)ZERO | ((uint32_t)ZERO << 16))) {
          const cd av = tr + asum;
          push(a, av * xb);
          push(b, av * xa);
        }
      }
    }
    for (int hc = 0; hc < 4; ++hc)
      if (F.hot_slot[hc] != ZERO) push(F.hot_slot[hc], hacc[hc]);
    if (full)
      for (const int4& ck : F.fw_ck) {
        if (ck.x < 0 || ck.x >= P1) return false;
        cd s = 0.0;
        for (int q = ck.y; q < ck.z; ++q) {
          const uint32_t en = F.fw_ent.at(q);
          s += ab.at(en & 0xffffu) * X(en >> 16);
        }
        ab.at(ck.x) += s;
      }
    phi[0] = accr.real();
    phi[1] = acci.imag();
    for (int i = 0; i < P1; ++i) {
      Abar[2 * i] = ab[i].real();
      Abar[2 * i + 1] = ab[i].imag();
    }
  } catch (const std::out_of_range&) {
    return false;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Rematerialising schedule (remat_kernel).  A term is a tuple of K of length
// >= 2, evaluated as the product of the two parents of its DAG node.  Rows
// are keyed by a parent; the entries of a row are (other parent,
// coefficient).  Forward only: a term sits in the row of its parent of
// larger order (on a tie, the parent that can head more rows).  With the
// adjoint: a term sits in the rows of both parents (a square once, with
// coefficient 2c).  Entries of one (row, order of the other parent) are cut
// into items of at most term_chunk; items of one (row order, other order)
// class are sorted by entry count and packed 64 to a slice, so every lane
// of a slice runs the same loops.
// ---------------------------------------------------------------------------
namespace {
struct REnt {
  int32_t row, oth, kmap, kbar;
};

// Factor lists of the other parents: the most frequent pairs of one-particle
// factors (counted over all entries) become pair slots P1 + 1 + r; each
// other parent takes disjoint pairs greedily over its sorted factors.
struct Factors {
  std::vector<int8_t> n;     // [V] factor count, -1 if the node is no other parent
  std::vector<uint64_t> lo, hi;
};

void compress_others(const HostGraph& h, const std::vector<REnt>& ents, int budget, ace_graph::Remat& R,
                     Factors& F) {
  const int P1 = h.P1, ONE = P1, W = h.width;
  const int64_t V = h.n_nodes();
  std::vector<int32_t> mult(V, 0);
  for (const REnt& e : ents) mult[e.oth] += 1;
  R.pairs.clear();
  std::vector<int32_t> pslot;
  if (budget > 0 && P1 <= 4096) {
    std::vector<int64_t> cnt((size_t)P1 * P1, 0);
    for (int64_t v = 0; v < V; ++v) {
      if (!mult[v] || h.node_len[v] < 2) continue;
      const int32_t* f = &h.node_flat[(size_t)v * W];
      const int L = h.node_len[v];
      for (int i = 0; i < L; ++i)
        for (int j = i + 1; j < L; ++j) cnt[(size_t)f[i] * P1 + f[j]] += mult[v];   // tuples are sorted
    }
    std::vector<int32_t> idx;
    for (size_t q = 0; q < cnt.size(); ++q)
      if (cnt[q] > 0) idx.push_back((int32_t)q);
    const size_t take = std::min<size_t>((size_t)budget, idx.size());
    std::partial_sort(idx.begin(), idx.begin() + take, idx.end(), [&](int32_t x, int32_t y) {
      return cnt[x] != cnt[y] ? cnt[x] > cnt[y] : x < y;
    });
    idx.resize(take);
    std::sort(idx.begin(), idx.end());
    pslot.assign((size_t)P1 * P1, -1);
    for (size_t r = 0; r < idx.size(); ++r) {
      pslot[idx[r]] = ONE + 1 + (int32_t)r;
      R.pairs.push_back((uint32_t)(idx[r] / P1) | ((uint32_t)(idx[r] % P1) << 16));
    }
  }
  F.n.assign(V, -1);
  F.lo.assign(V, 0);
  F.hi.assign(V, 0);
  for (int64_t v = 0; v < V; ++v) {
    if (!mult[v]) continue;
    const int32_t* f = &h.node_flat[(size_t)v * W];
    const int L = h.node_len[v];
    int out[8], no = 0;
    bool used[8] = {false, false, false, false, false, false, false, false};
    if (!pslot.empty())
      for (int i = 0; i < L; ++i) {
        if (used[i]) continue;
        for (int j = i + 1; j < L; ++j)
          if (!used[j] && pslot[(size_t)f[i] * P1 + f[j]] >= 0) {
            used[i] = used[j] = true;
            out[no++] = pslot[(size_t)f[i] * P1 + f[j]];
            break;
          }
      }
    for (int i = 0; i < L; ++i)
      if (!used[i]) out[no++] = f[i];
    uint64_t lo = 0, hi = 0;
    for (int u = 0; u < 8; ++u) {
      const uint64_t sl = 16 * (u < no ? (uint64_t)out[u] : (uint64_t)ONE);   // LDS byte offset
      (u < 4 ? lo : hi) |= sl << (16 * (u & 3));
    }
    F.n[v] = (int8_t)no;
    F.lo[v] = lo;
    F.hi[v] = hi;
  }
}

// Pair slots that fit beside the one-particle values (and adjoints) of the
// block's environments without lowering the number of resident waves below
// what the kernel's registers allow: remat_kernel<true> holds 4 waves per
// SIMD, <false> 5 (gfx950, 512 VGPRs per lane, at most 128 per lane at the
// kernel's 1024-thread bound), i.e. 16 and 20 waves per CU of 160 KiB LDS.
int auto_pair_slots(const ace_graph* g, bool grad) {
  const int ne = std::max(1, g->opts.env_per_block);
  const int wave_per_block = std::max(1, g->opts.block_threads / 64);
  const int waves_cu = grad ? 16 : 20;
  const int blocks = std::max(1, waves_cu / wave_per_block);
  const size_t per_block = (size_t)160 * 1024 / blocks;
  const size_t base = (size_t)ne * (g->P1 + 1) * 16 * (grad ? 2 : 1) + 16 * 16 + 256;
  return per_block > base ? (int)std::min<size_t>(8192, (per_block - base) / (16 * (size_t)ne)) : 0;
}

void pack_remat(ace_graph* g, std::vector<REnt>& ents, ace_graph::Remat& R, bool grad) {
  const HostGraph& h = g->h;
  const int P1 = h.P1, ONE = P1, W = h.width;
  Factors F;
  const int budget = g->opts.pair_slots >= 0 ? g->opts.pair_slots : auto_pair_slots(g, grad);
  compress_others(h, ents, std::max(0, std::min(budget, kRematMaxSlots - P1 - 1)), R, F);
  R.slice.clear();
  R.rlo.clear();
  R.rhi.clear();
  R.olo.clear();
  R.ohi.clear();
  R.kmap.assign(P1, -1);
  for (int i = 0; i < P1; ++i) R.kmap[i] = h.node_k[i];
  R.kbar.clear();
  if (R.fold) R.kbar.assign(P1, -1);   // tuples of length one in K have m = 0: self-conjugate
  R.cs_leaf = 0;
  R.cs_ent = P1;
  std::stable_sort(ents.begin(), ents.end(), [&](const REnt& x, const REnt& y) {
    if (x.row != y.row) return x.row < y.row;
    const int sx = F.n[x.oth], sy = F.n[y.oth];
    if (sx != sy) return sx < sy;
    return x.oth < y.oth;
  });
  struct Item {
    int32_t row;
    int nb, sig;
    int64_t first;
    int count, chunk;
  };
  std::vector<Item> items;
  const int C = std::max(1, g->opts.term_chunk);
  for (size_t i = 0; i < ents.size();) {
    size_t j = i;
    const int sig = F.n[ents[i].oth];
    while (j < ents.size() && ents[j].row == ents[i].row && F.n[ents[j].oth] == sig) ++j;
    int chunk = 0;
    for (size_t c0 = i; c0 < j; c0 += C)
      items.push_back({ents[i].row, (int)h.node_len[ents[i].row], sig, (int64_t)c0, (int)std::min<size_t>(C, j - c0),
                       chunk++});
    i = j;
  }
  // chunks of one row go to different slices where possible: their adjoint
  // pushes hit the same addresses, which a wave would serialise
  // items of equal shape and length in a hashed order: neighbouring rows in
  // node order share factors, and rows that share a factor in one slice push
  // to one address (same-address LDS atomics in one instruction serialise)
  auto mix = [](uint64_t v) {
    v += 0x9e3779b97f4a7c15ull;
    v = (v ^ (v >> 30)) * 0xbf58476d1ce4e5b9ull;
    v = (v ^ (v >> 27)) * 0x94d049bb133111ebull;
    return v ^ (v >> 31);
  };
  std::stable_sort(items.begin(), items.end(), [&](const Item& x, const Item& y) {
    if (x.nb != y.nb) return x.nb < y.nb;
    if (x.sig != y.sig) return x.sig < y.sig;
    if (x.count != y.count) return x.count > y.count;
    const uint64_t hx = mix(((uint64_t)(uint32_t)x.row << 16) | (uint32_t)x.chunk);
    const uint64_t hy = mix(((uint64_t)(uint32_t)y.row << 16) | (uint32_t)y.chunk);
    if (hx != hy) return hx < hy;
    return x.chunk < y.chunk;
  });
  // hot one-particle slots: the most frequent adjoint push targets
  {
    std::vector<int64_t> freq(P1 + 1, 0);
    int64_t npush = 0;
    for (const Item& it : items)
      for (int u = 0; u < it.nb; ++u) {
        freq[h.node_flat[(int64_t)it.row * W + u]] += 1;
        ++npush;
      }
    std::vector<int32_t> ord(P1);
    for (int i = 0; i < P1; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return freq[x] > freq[y]; });
    for (int k = 0; k < 4; ++k)
      R.hot[k] = (k < g->opts.hot_columns && k < P1 && freq[ord[k]] * 64 >= npush) ? ord[k] : ONE;
  }
  // factors of a row node in the order perm (factor perm[u] at position u):
  // lanes of a slice order their factor lists differently, so rows that
  // share factors do not push to one address, or one bank pair, in one
  // instruction (the product does not depend on the order)
  using Perm = std::array<int8_t, 8>;
  auto pack = [&](int32_t node, int from, const Perm& perm) {
    const int count = h.node_len[node];
    uint64_t w = 0;
    for (int u = 0; u < 4; ++u) {
      const int idx = from + u;
      const uint64_t sl =
          16 * (idx < count ? (uint64_t)h.node_flat[(int64_t)node * W + perm[idx]] : (uint64_t)ONE);
      w |= sl << (16 * u);
    }
    return w;
  };
  // the factor orders tried for a row of nb factors: every permutation up to
  // five factors, else the rotations
  auto perms_of = [](int nb) {
    std::vector<Perm> ps;
    Perm pm{};
    for (int u = 0; u < 8; ++u) pm[u] = (int8_t)u;
    if (nb <= 5) {
      do ps.push_back(pm);
      while (std::next_permutation(pm.begin(), pm.begin() + nb));
    } else {
      for (int r = 0; r < nb; ++r) {
        Perm rp{};
        for (int u = 0; u < 8; ++u) rp[u] = (int8_t)(u < nb ? (u + r) % nb : u);
        ps.push_back(rp);
      }
    }
    return ps;
  };
  const uint64_t one16 = 16 * (uint64_t)ONE;
  const uint64_t ones = one16 | (one16 << 16) | (one16 << 32) | (one16 << 48);
  // Slices of 64 lanes.  Within each group of equal (nb, sig), the items
  // (in the order above) go to one of a few open slices: the one, and the
  // factor rotation, where the item's row pushes add the least LDS atomic
  // contention to the slice's push instructions so far.  Push i of every
  // lane goes to factor i of its rotated row list.  The LDS serves the
  // 8-byte atomics of a push a quarter-wave at a time over 16 bank pairs;
  // with the adjoints in Re and Im planes a lane's atomic lands on pair
  // slot mod 16 (up to a shift), and the cost is set by the most lanes on
  // one pair; lanes on one address serialise as well.  The hot slots, summed
  // in registers, and the constant slot do not count.  A slice is emitted when full; its first
  // item is its longest, since the items come longest first.
  std::vector<Item> ordered;
  std::vector<Perm> item_perm;
  std::vector<size_t> cut;   // slice ends in `ordered`
  {
    constexpr int kOpen = 4;
    struct Open {
      std::vector<size_t> idx;
      std::vector<Perm> perm;
      std::vector<std::map<int32_t, int>> mult;   // per push: lanes on a slot, keyed 4 * slot + quarter
      std::vector<std::array<int, 64>> bank;       // per push: lanes on a bank pair, [16 * quarter + slot mod 16]
    };
    const int nh = std::min(g->opts.hot_columns, g->opts.env_per_block > 1 ? 2 : 4);
    auto is_hot = [&](int32_t sl) {
      if (sl == ONE) return true;
      for (int k = 0; k < nh; ++k)
        if (sl == R.hot[k]) return true;
      return false;
    };
    ordered.reserve(items.size());
    item_perm.reserve(items.size());
    for (size_t g0 = 0; g0 < items.size();) {
      size_t g1 = g0;
      while (g1 < items.size() && items[g1].nb == items[g0].nb && items[g1].sig == items[g0].sig) ++g1;
      const int nbs = items[g0].nb;
      const std::vector<Perm> perms = perms_of(nbs);
      std::vector<Open> open(kOpen);
      auto reset = [&](Open& o) {
        o.idx.clear();
        o.perm.clear();
        o.mult.assign(nbs, {});
        o.bank.assign(nbs, {});
        for (auto& bk : o.bank) bk.fill(0);
      };
      auto flush = [&](Open& o) {
        for (size_t t = 0; t < o.idx.size(); ++t) {
          ordered.push_back(items[o.idx[t]]);
          item_perm.push_back(o.perm[t]);
        }
        cut.push_back(ordered.size());
        reset(o);
      };
      for (auto& o : open) reset(o);
      for (size_t t = g0; t < g1; ++t) {
        const int32_t* f = &h.node_flat[(int64_t)items[t].row * W];
        int bs = 0, bc = INT32_MAX;
        size_t bp = 0;
        for (int k = 0; k < kOpen && bc > 0; ++k) {
          const int lane = (int)open[k].idx.size();
          const int quarter = lane >> 4;
          int col[8][8];   // col[i][u]: contention of factor u pushed at position i
          for (int i = 0; i < nbs; ++i)
            for (int u = 0; u < nbs; ++u) {
              const int32_t sl = f[u];
              col[i][u] = 0;
              if (is_hot(sl)) continue;
              const auto m = open[k].mult[i].find(4 * sl + quarter);
              col[i][u] = (m == open[k].mult[i].end() ? 0 : m->second) + open[k].bank[i][16 * quarter + (sl & 15)];
            }
          // start the scan at a lane-dependent order: among equal costs,
          // neighbouring lanes take different orders
          for (size_t q0 = 0; q0 < perms.size(); ++q0) {
            const size_t q = (q0 + (size_t)lane) % perms.size();
            int cost = 0;
            for (int i = 0; i < nbs; ++i) cost += col[i][perms[q][i]];
            if (cost < bc) {
              bc = cost;
              bs = k;
              bp = q;
              if (cost == 0) break;
            }
          }
        }
        Open& o = open[bs];
        const Perm& pm = perms[bp];
        const int quarter = (int)o.idx.size() >> 4;
        for (int i = 0; i < nbs; ++i) {
          const int32_t sl = f[pm[i]];
          if (is_hot(sl)) continue;
          o.mult[i][4 * sl + quarter] += 1;
          o.bank[i][16 * quarter + (sl & 15)] += 1;
        }
        o.idx.push_back(t);
        o.perm.push_back(pm);
        if (o.idx.size() == 64) flush(o);
      }
      for (auto& o : open)
        if (!o.idx.empty()) flush(o);
      g0 = g1;
    }
  }
  int64_t pos = 0;
  size_t i0 = 0;
  for (const size_t i1 : cut) {
    const std::vector<Item>& items = ordered;   // the emission below reads the slice order
    const int ncol = items[i0].count;
    if ((int64_t)R.rlo.size() + 64 > INT32_MAX || P1 + pos + 64LL * ncol > kRematMaxEntries)
      throw std::length_error("remat schedule larger than 2^26 entries");
    const int sig = items[i0].sig;
    R.slice.push_back(make_int4((int)R.rlo.size(), (int)pos, ncol, items[i0].nb | (sig << 8)));
    const size_t e0 = R.olo.size();
    R.olo.resize(e0 + 64 * (size_t)ncol, ones);
    R.ohi.resize(e0 + 64 * (size_t)ncol, ones);
    R.kmap.resize(P1 + e0 + 64 * (size_t)ncol, -1);
    if (R.fold) R.kbar.resize(P1 + e0 + 64 * (size_t)ncol, -1);
    // per lane: its entries, then their column and factor rotation
    std::vector<std::vector<int64_t>> lane_ents(64);
    for (int lane = 0; lane < 64; ++lane) {
      if (i0 + lane < i1) {
        const Item& it = items[i0 + lane];
        R.rlo.push_back(pack(it.row, 0, item_perm[i0 + lane]));
        R.rhi.push_back(pack(it.row, 4, item_perm[i0 + lane]));
        for (int j = 0; j < it.count; ++j) lane_ents[lane].push_back(it.first + j);
      } else {
        R.rlo.push_back(ones);
        R.rhi.push_back(ones);
      }
    }
    auto factor = [&](int64_t ei, int u) {
      const int32_t o = ents[ei].oth;
      return (int)(((u < 4 ? F.lo[o] : F.hi[o]) >> (16 * (u & 3))) & 0xffffu);
    };
    // entry ei with factor perm[u] read at position u
    auto put_entry = [&](int lane, int j, int64_t ei, const int* perm) {
      const size_t e = e0 + (size_t)j * 64 + lane;
      uint64_t lo = 0, hi = 0;
      for (int u = 0; u < 8; ++u) {
        const uint64_t sl = u < sig ? (uint64_t)factor(ei, perm[u]) : one16;
        (u < 4 ? lo : hi) |= sl << (16 * (u & 3));
      }
      R.olo[e] = lo;
      R.ohi[e] = hi;
      R.kmap[P1 + e] = ents[ei].kmap;
      if (R.fold) R.kbar[P1 + e] = ents[ei].kbar;
    };
    const int ident[8] = {0, 1, 2, 3, 4, 5, 6, 7};
    if (!g->opts.bank_schedule) {
      for (int lane = 0; lane < 64; ++lane)
        for (size_t j = 0; j < lane_ents[lane].size(); ++j) put_entry(lane, (int)j, lane_ents[lane][j], ident);
    } else {
      // Greedy per column and quarter-wave: each lane takes the remaining
      // entry and order of its factors (any permutation up to five factors,
      // else a rotation: the product does not depend on it) that adds the
      // fewest 16-byte bank-group collisions (slot mod 16) over the factor
      // reads of that column; a slot already read in the quarter is a
      // broadcast and costs nothing.
      std::vector<std::array<int8_t, 8>> perms;
      {
        std::array<int8_t, 8> pm{};
        for (int u = 0; u < 8; ++u) pm[u] = (int8_t)u;
        if (sig <= 5) {
          do perms.push_back(pm);
          while (std::next_permutation(pm.begin(), pm.begin() + sig));
        } else {
          for (int r = 0; r < sig; ++r) {
            std::array<int8_t, 8> rp{};
            for (int u = 0; u < 8; ++u) rp[u] = (int8_t)(u < sig ? (u + r) % sig : u);
            perms.push_back(rp);
          }
        }
      }
      for (int q = 0; q < 4; ++q)
        for (int j = 0; j < ncol; ++j) {
          int16_t seen[8][16];   // per factor position and bank group: a slot read there, or -1 (-2: several)
          for (auto& r : seen)
            for (auto& v : r) v = -1;
          for (int lane = 16 * q; lane < 16 * q + 16; ++lane) {
            auto& L = lane_ents[lane];
            if (L.empty()) continue;
            int best = 0, best_cost = INT32_MAX;
            size_t best_p = 0;
            const int ncand = std::min<int>((int)L.size(), 24);
            for (int c = 0; c < ncand && best_cost > 0; ++c) {
              int8_t col[8][8];   // col[u][t]: factor t read at position u collides
              for (int u = 0; u < sig; ++u)
                for (int t = 0; t < sig; ++t) {
                  const int sl = factor(L[c], t) >> 4;
                  const int16_t v = seen[u][sl & 15];
                  col[u][t] = (v != -1 && v != sl) ? 1 : 0;
                }
              for (size_t pi = 0; pi < perms.size(); ++pi) {
                int cost = 0;
                for (int u = 0; u < sig; ++u) cost += col[u][perms[pi][u]];
                if (cost < best_cost) {
                  best_cost = cost;
                  best = c;
                  best_p = pi;
                  if (cost == 0) break;
                }
              }
            }
            const int64_t ei = L[best];
            L.erase(L.begin() + best);
            int perm[8];
            for (int u = 0; u < 8; ++u) perm[u] = perms[best_p][u];
            for (int u = 0; u < sig; ++u) {
              const int sl = factor(ei, perm[u]) >> 4;
              int16_t& v = seen[u][sl & 15];
              v = (v == -1 || v == sl) ? (int16_t)sl : (int16_t)-2;
            }
            put_entry(lane, j, ei, perm);
          }
        }
    }
    pos += 64LL * ncol;
    i0 = i1;
  }
  R.nslices = (int)R.slice.size();
  R.nitems = (int)R.rlo.size();
}
}  // namespace

// Conjugate partner of every tuple of K: the tuple with every m negated
// (x_kbar = conj(x_k) when A_{n,l,-m} = (-1)^m conj(A_{n,l,m}) and the
// m of k sum to zero).  K is sorted lexicographically within each length,
// so the partner is found by binary search.
std::vector<int64_t> conj_partners(const HostGraph& h) {
  const int P1 = h.P1, W = h.width;
  std::vector<int32_t> cj(P1, -1);
  for (int i = 0; i < P1; ++i)
    for (int j = 0; j < P1; ++j)
      if (h.on_n[j] == h.on_n[i] && h.on_l[j] == h.on_l[i] && h.on_m[j] == -h.on_m[i] && h.on_k[j] == h.on_k[i]) {
        cj[i] = j;
        break;
      }
  for (int i = 0; i < P1; ++i)
    if (cj[i] < 0) throw std::logic_error("one-particle set not closed under m -> -m");
  std::vector<int64_t> out(h.nK, -1);
  int64_t first[9] = {0};
  for (int nu = 1; nu <= 8; ++nu) first[nu] = first[nu - 1] + (nu - 1 >= 1 ? h.nK_by_order[nu - 1] : 0);
  for (int64_t q = 0; q < h.nK; ++q) {
    const int L = h.k_len[q];
    int32_t t[8];
    for (int u = 0; u < L; ++u) t[u] = cj[h.k_flat[(size_t)q * W + u]];
    std::sort(t, t + L);
    int64_t lo = first[L], hi = first[L] + h.nK_by_order[L];
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      const int32_t* r = &h.k_flat[(size_t)mid * W];
      if (std::lexicographical_compare(r, r + L, t, t + L))
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo >= first[L] + h.nK_by_order[L] || !std::equal(t, t + L, &h.k_flat[(size_t)lo * W]))
      throw std::logic_error("K not closed under m -> -m");
    out[q] = lo;
  }
  return out;
}

void make_remat(ace_graph* g) {
  const HostGraph& h = g->h;
  const int P1 = h.P1;
  const int64_t V = h.n_nodes();
  g->remat_ok = false;
  if (P1 + 1 > kRematMaxSlots) {
    g->remat_why = "more than 4095 one-particle functions";
    return;
  }
  if (h.width > 8) {
    g->remat_why = "correlation order above 8";
    return;
  }
  std::vector<int32_t> tie(V, 0);
  for (int64_t q = 0; q < h.nK; ++q) {
    if (h.k_len[q] < 2) continue;
    const int64_t v = h.k_to_node[q];
    const int32_t a = h.par[2 * v], b = h.par[2 * v + 1];
    if (h.node_len[a] == h.node_len[b]) {
      tie[a] += 1;
      tie[b] += 1;
    }
  }
  const std::vector<int64_t> kbar = conj_partners(h);
  for (int f = 0; f < 2; ++f) {
    std::vector<REnt> one, two;
    one.reserve((size_t)h.nK);
    two.reserve(2 * (size_t)h.nK);
    for (int64_t q = 0; q < h.nK; ++q) {
      if (h.k_len[q] < 2) continue;
      int32_t kb = -1;
      if (f) {
        if (kbar[q] < q) continue;   // the partner with the smaller index carries the pair
        kb = kbar[q] == q ? -1 : (int32_t)kbar[q];
      }
      const int64_t v = h.k_to_node[q];
      const int32_t a = h.par[2 * v], b = h.par[2 * v + 1];
      const int la = h.node_len[a], lb = h.node_len[b];
      const bool a_row = la > lb || (la == lb && tie[a] >= tie[b]);
      one.push_back({a_row ? a : b, a_row ? b : a, (int32_t)q, kb});
      if (a == b) {
        two.push_back({a, a, -2 - (int32_t)q, kb});   // M_aa = 2 c
      } else {
        two.push_back({a, b, (int32_t)q, kb});
        two.push_back({b, a, (int32_t)q, kb});
      }
    }
    g->rm[2 * f].fold = g->rm[2 * f + 1].fold = f == 1;
    try {
      pack_remat(g, one, g->rm[2 * f], false);
      pack_remat(g, two, g->rm[2 * f + 1], true);
    } catch (const std::length_error& e) {
      g->remat_why = e.what();
      return;
    }
  }
  g->remat_ok = true;
  g->remat_why.clear();
}

// Host run of a remat schedule for one environment (grad: the two-sided
// one), with the kernel's indices, padding and push order; false if an
// index is out of range.
bool remat_emulate(const ace_graph* g, int which, const double* coeffs, const double* A, double* phi, double* Abar) {
  using cd = std::complex<double>;
  const ace_graph::Remat& R = g->rm[which];
  const bool grad = which & 1;
  const int P1 = g->P1, ONE = P1;
  // (Re weight, Im weight) of every coefficient position
  std::vector<double> cs(R.kmap.size()), cs2(R.kmap.size());
  for (size_t i = 0; i < cs.size(); ++i) {
    const int k = R.kmap[i];
    if (k == -1) continue;
    const int q = k >= 0 ? k : -2 - k;
    const double sc = k >= 0 ? 1.0 : 2.0;
    const int kb = R.fold ? R.kbar[i] : -1;
    cs[i] = sc * (kb >= 0 ? coeffs[q] + coeffs[kb] : coeffs[q]);
    cs2[i] = sc * (kb >= 0 ? coeffs[q] - coeffs[kb] : coeffs[q]);
  }
  const int NP = (int)R.pairs.size();
  std::vector<cd> x(P1 + 1 + NP), ab(P1 + 1);
  for (int i = 0; i < P1; ++i) {
    x[i] = cd(A[2 * i], A[2 * i + 1]);
    ab[i] = cs[R.cs_leaf + i];
  }
  x[ONE] = 1.0;
  for (int r = 0; r < NP; ++r) {
    const int a = (int)(R.pairs[r] & 0xffffu), b = (int)(R.pairs[r] >> 16);
    if (a >= P1 || b >= P1) return false;
    x[ONE + 1 + r] = x[a] * x[b];
  }
  double acc_re = 0.0, acc_im = 0.0;
  for (int i = 0; i < P1; ++i) {
    acc_re += cs[R.cs_leaf + i] * x[i].real();
    acc_im += cs2[R.cs_leaf + i] * x[i].imag();
  }
  auto ok = [&](int v) { return v >= 0 && v <= P1 + NP; };
  auto okrow = [&](int v) { return v >= 0 && v <= P1; };
  auto slot = [](uint64_t lo, uint64_t hi, int i) {   // fields are LDS byte offsets of 16-byte slots
    return (int)((((i < 4 ? lo : hi) >> (16 * (i & 3))) & 0xffffu) >> 4);
  };
  for (const int4& sl : R.slice) {
    const int nb = sl.w & 0xff, sig = sl.w >> 8;
    if (nb < 1 || nb > 8 || sig < 1 || sig > 7) return false;
    for (int lane = 0; lane < 64; ++lane) {
      const int item = sl.x + lane;
      if (item < 0 || item >= R.nitems) return false;
      cd xb = 1.0;
      for (int i = 0; i < nb; ++i) {
        const int v = slot(R.rlo[item], R.rhi[item], i);
        if (!okrow(v)) return false;
        xb = i == 0 ? x[v] : xb * x[v];
      }
      cd y = 0.0, y2 = 0.0;
      for (int j = 0; j < sl.z; ++j) {
        const int64_t pos = (int64_t)sl.y + (int64_t)j * 64 + lane;
        if (pos < 0 || pos >= (int64_t)R.olo.size()) return false;
        cd xo = 1.0;
        for (int u = 0; u < sig; ++u) {
          const int v = slot(R.olo[pos], R.ohi[pos], u);
          if (!ok(v)) return false;
          xo = u == 0 ? x[v] : xo * x[v];
        }
        y += cs[R.cs_ent + pos] * xo;
        y2 += cs2[R.cs_ent + pos] * xo;
      }
      const double w = grad ? 0.5 : 1.0;
      acc_re += w * (xb * y).real();
      acc_im += w * (xb * y2).imag();
      if (!grad) continue;
      if (slot(R.rlo[item], R.rhi[item], 0) != ONE)
        for (int i = 0; i < nb; ++i) {
          cd d = y;
          for (int w = 0; w < nb; ++w)
            if (w != i) d *= x[slot(R.rlo[item], R.rhi[item], w)];
          ab[slot(R.rlo[item], R.rhi[item], i)] += d;
        }
    }
  }
  phi[0] = acc_re;
  phi[1] = acc_im;
  if (Abar)
    for (int i = 0; i < P1; ++i) {
      Abar[2 * i] = ab[i].real();
      Abar[2 * i + 1] = ab[i].imag();
    }
  return true;
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

// LDS of forest_kernel: values of every resident slot, one-particle
// adjoints (reverse pass), the order-2 parent table, reduction scratch.
size_t forest_lds_bytes(const ace_graph::Forest& F, int P1, bool grad, bool full, int ne = 1) {
  size_t b = (size_t)F.nslot * 16;
  if (grad && full) b += (size_t)F.nslot * 16;
  if (grad && !full) b += (size_t)(P1 + 1) * 16;
  b *= (size_t)ne;
  if (grad && !full) b += ((size_t)F.N2 * 4 + 15) / 16 * 16;
  return b + (kForestThreads / 64) * sizeof(double2);
}

// forest_kernel variants: [environments per block - 1][folded][forward /
// reverse with one-particle adjoints / reverse with every resident
// adjoint][grandchildren]
using ForestKernel = void (*)(ForestArgs);
template <int NE, bool FOLD>
constexpr ForestKernel forest_row[3][2] = {
    {forest_kernel<false, false, false, FOLD, NE>, forest_kernel<false, true, false, FOLD, NE>},
    {forest_kernel<true, false, false, FOLD, NE>, forest_kernel<true, true, false, FOLD, NE>},
    {forest_kernel<true, false, true, FOLD, NE>, forest_kernel<true, true, true, FOLD, NE>}};

ForestKernel forest_variant(int ne, bool fold, int mode, bool gc) {
  const int g = gc ? 1 : 0;
  if (ne == 2) return fold ? forest_row<2, true>[mode][g] : forest_row<2, false>[mode][g];
  return fold ? forest_row<1, true>[mode][g] : forest_row<1, false>[mode][g];
}

std::vector<const void*> forest_variants() {
  std::vector<const void*> v;
  for (int ne = 1; ne <= 2; ++ne)
    for (int f = 0; f < 2; ++f)
      for (int mode = 0; mode < 3; ++mode)
        for (int gc = 0; gc < 2; ++gc) v.push_back((const void*)forest_variant(ne, f == 1, mode, gc == 1));
  return v;
}

template <typename T>
T* carve(char*& p, size_t n) {
  T* r = reinterpret_cast<T*>(p);
  p += align_up(n * sizeof(T));
  return r;
}

// LDS of remat_kernel: one-particle values and adjoints, reduction scratch.
size_t remat_lds_bytes(const ace_graph* g, int which, int ne = 1) {
  const bool grad = which & 1;
  const size_t np = g->rm[which].pairs.size();
  return (size_t)ne * ((g->P1 + 1 + np) * 16 + (grad ? (size_t)(g->P1 + 1) * 16 : 0)) +
         (kRematBlock / 64) * sizeof(double2);
}

// Environments one remat block evaluates: the requested number where their
// values fit in LDS, else one.
int remat_env_per_block(const ace_graph* g, int which) {
  return g->opts.env_per_block >= 2 && remat_lds_bytes(g, which, 2) <= g->max_lds ? 2 : 1;
}

// Block size of the forest kernel (its schedule spreads over at most
// kMaxForestWaves waves).
int forest_threads(const ace_graph* g) { return std::min(g->opts.block_threads, 64 * kMaxForestWaves); }

// Upload the forest and remat schedules (replacing previous ones) and plan
// their LDS.
ace_status upload_forest(ace_graph* g) {
  if (g->fmem) {
    (void)hipFree(g->fmem);
    g->fmem = nullptr;
  }
  auto put = [](void* d, const void* s, size_t n) { return n ? hipMemcpy(d, s, n, hipMemcpyHostToDevice) : hipSuccess; };
  const int maxl = (int)g->max_lds;
  size_t fb = kAlign;
  for (const ace_graph::Forest& F : g->fo) {
    if (!F.ok) continue;
    fb += align_up(F.nu2_ab.size() * 4) + align_up(F.it_ab.size() * 4);
    fb += align_up(F.mr_slice.size() * sizeof(int4)) + align_up(F.tr_slice.size() * sizeof(int4));
    fb += align_up(F.mr_row.size() * 2) + align_up(F.me_col.size() * 2) + align_up(F.ch_s.size() * 2);
    fb += align_up(F.gc_s.size() * 2) + align_up(F.ch_g.size() * sizeof(int2)) + align_up(F.kmap.size() * 4);
    fb += align_up(F.kbar.size() * 4) + align_up(F.fw_ck.size() * sizeof(int4)) + align_up(F.fw_ent.size() * 4);
  }
  if (g->fo[0].ok || g->fo[1].ok) {
    if (hipMalloc(&g->fmem, fb) != hipSuccess) {
      g->fmem = nullptr;
      (void)hipGetLastError();
      return fail(ACE_ERR_OUT_OF_MEMORY, "hipMalloc of the forest schedule failed");
    }
    char* q = static_cast<char*>(g->fmem);
    for (ace_graph::Forest& F : g->fo) {
      if (!F.ok) continue;
      F.d_nu2_ab = carve<uint32_t>(q, F.nu2_ab.size());
      F.d_it_ab = carve<uint32_t>(q, F.it_ab.size());
      F.d_mr_slice = carve<int4>(q, F.mr_slice.size());
      F.d_tr_slice = carve<int4>(q, F.tr_slice.size());
      F.d_mr_row = carve<uint16_t>(q, F.mr_row.size());
      F.d_me_col = carve<uint16_t>(q, F.me_col.size());
      F.d_ch_s = carve<uint16_t>(q, F.ch_s.size());
      F.d_gc_s = carve<uint16_t>(q, F.gc_s.size());
      F.d_ch_g = carve<int2>(q, F.ch_g.size());
      F.d_kmap = carve<int32_t>(q, F.kmap.size());
      F.d_kbar = carve<int32_t>(q, F.kbar.size());
      F.d_fw_ck = carve<int4>(q, F.fw_ck.size());
      F.d_fw_ent = carve<uint32_t>(q, F.fw_ent.size());
      ACE_HIP(put(F.d_nu2_ab, F.nu2_ab.data(), F.nu2_ab.size() * 4));
      ACE_HIP(put(F.d_it_ab, F.it_ab.data(), F.it_ab.size() * 4));
      ACE_HIP(put(F.d_mr_slice, F.mr_slice.data(), F.mr_slice.size() * sizeof(int4)));
      ACE_HIP(put(F.d_tr_slice, F.tr_slice.data(), F.tr_slice.size() * sizeof(int4)));
      ACE_HIP(put(F.d_mr_row, F.mr_row.data(), F.mr_row.size() * 2));
      ACE_HIP(put(F.d_me_col, F.me_col.data(), F.me_col.size() * 2));
      ACE_HIP(put(F.d_ch_s, F.ch_s.data(), F.ch_s.size() * 2));
      ACE_HIP(put(F.d_gc_s, F.gc_s.data(), F.gc_s.size() * 2));
      ACE_HIP(put(F.d_ch_g, F.ch_g.data(), F.ch_g.size() * sizeof(int2)));
      ACE_HIP(put(F.d_kmap, F.kmap.data(), F.kmap.size() * 4));
      ACE_HIP(put(F.d_kbar, F.kbar.data(), F.kbar.size() * 4));
      ACE_HIP(put(F.d_fw_ck, F.fw_ck.data(), F.fw_ck.size() * sizeof(int4)));
      ACE_HIP(put(F.d_fw_ent, F.fw_ent.data(), F.fw_ent.size() * 4));
      F.fwd_lds = forest_lds_bytes(F, g->P1, false, false) <= g->max_lds;
      F.full = forest_lds_bytes(F, g->P1, true, true) <= g->max_lds;
      F.grad_lds = F.full || forest_lds_bytes(F, g->P1, true, false) <= g->max_lds;
    }
    for (const void* f : forest_variants())
      ACE_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  }
  if (g->rmem) {
    (void)hipFree(g->rmem);
    g->rmem = nullptr;
  }
  g->remat_lds = false;
  if (g->remat_ok) {
    size_t rb = kAlign;
    for (const auto& R : g->rm)
      rb += align_up(R.slice.size() * sizeof(int4)) + align_up(R.rlo.size() * 8) + align_up(R.rhi.size() * 8) +
            align_up(R.olo.size() * 8) + align_up(R.ohi.size() * 8) + align_up(R.kmap.size() * 4) +
            align_up(R.pairs.size() * 4) + align_up(R.kbar.size() * 4);
    if (hipMalloc(&g->rmem, rb) != hipSuccess) {
      g->rmem = nullptr;
      (void)hipGetLastError();
      return fail(ACE_ERR_OUT_OF_MEMORY, "hipMalloc of the remat schedule failed");
    }
    char* q = static_cast<char*>(g->rmem);
    for (auto& R : g->rm) {
      R.d_slice = carve<int4>(q, R.slice.size());
      R.d_rlo = carve<uint64_t>(q, R.rlo.size());
      R.d_rhi = carve<uint64_t>(q, R.rhi.size());
      R.d_olo = carve<uint64_t>(q, R.olo.size());
      R.d_ohi = carve<uint64_t>(q, R.ohi.size());
      R.d_kmap = carve<int32_t>(q, R.kmap.size());
      R.d_pairs = carve<uint32_t>(q, R.pairs.size());
      R.d_kbar = carve<int32_t>(q, R.kbar.size());
      ACE_HIP(put(R.d_pairs, R.pairs.data(), R.pairs.size() * 4));
      ACE_HIP(put(R.d_kbar, R.kbar.data(), R.kbar.size() * 4));
      ACE_HIP(put(R.d_slice, R.slice.data(), R.slice.size() * sizeof(int4)));
      ACE_HIP(put(R.d_rlo, R.rlo.data(), R.rlo.size() * 8));
      ACE_HIP(put(R.d_rhi, R.rhi.data(), R.rhi.size() * 8));
      ACE_HIP(put(R.d_olo, R.olo.data(), R.olo.size() * 8));
      ACE_HIP(put(R.d_ohi, R.ohi.data(), R.ohi.size() * 8));
      ACE_HIP(put(R.d_kmap, R.kmap.data(), R.kmap.size() * 4));
    }
    g->remat_lds = true;
    for (int which = 0; which < 4; ++which) g->remat_lds &= remat_lds_bytes(g, which) <= g->max_lds;
    const void* rk[] = {
        (const void*)remat_kernel<false, false, 1, false>, (const void*)remat_kernel<true, false, 1, false>,
        (const void*)remat_kernel<false, true, 1, false>,  (const void*)remat_kernel<true, true, 1, false>,
        (const void*)remat_kernel<false, false, 2, false>, (const void*)remat_kernel<true, false, 2, false>,
        (const void*)remat_kernel<false, true, 2, false>,  (const void*)remat_kernel<true, true, 2, false>,
        (const void*)remat_kernel<false, false, 1, true>,  (const void*)remat_kernel<true, false, 1, true>,
        (const void*)remat_kernel<false, true, 1, true>,   (const void*)remat_kernel<true, true, 1, true>,
        (const void*)remat_kernel<false, false, 2, true>,  (const void*)remat_kernel<true, false, 2, true>,
        (const void*)remat_kernel<false, true, 2, true>,   (const void*)remat_kernel<true, true, 2, true>};
    for (const void* f : rk) ACE_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  }
  return ACE_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device), looked up
// once per device.
ace_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ACE_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(ACE_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return ACE_OK;
}

ace_status upload(ace_graph* g) {
  int dev = 0;
  ACE_HIP(hipGetDevice(&dev));
  g->device = dev;
  {
    // the fixed workspace of ace_eval_grad_noalloc is located on every
    // device a graph is built on
    void* unused = nullptr;
    const ace_status sst = scratch_address(dev, &unused);
    if (sst != ACE_OK) return sst;
  }
  int lds = 0;
  ACE_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  g->max_lds = (size_t)lds;
  size_t bytes = 0;
  bytes += align_up(g->st_ab.size() * sizeof(int2)) + align_up(g->st_k.size() * 4);
  bytes += align_up(g->cl_ab.size() * sizeof(int2)) + align_up(g->cl_k.size() * 4);
  bytes += align_up(g->leaf_k.size() * 4) + align_up(g->nv_idx.size() * 2) + align_up(g->nv_kmap.size() * 4);
  bytes += align_up(g->nv_slice.size() * sizeof(int4));
  bytes += align_up(g->onep.size() * sizeof(OnepInfo)) + align_up(g->onep_index.size() * 2);
  bytes += align_up(g->basis_prim.size() * 2);
  bytes += align_up(g->ycoef.size() * 8) + align_up(g->gsrc.size() * 4) + kAlign;
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
  g->d_nv_idx = carve<int16_t>(p, g->nv_idx.size());
  g->d_nv_kmap = carve<int32_t>(p, g->nv_kmap.size());
  g->d_nv_slice = carve<int4>(p, g->nv_slice.size());
  g->d_onep = carve<OnepInfo>(p, g->onep.size());
  g->d_onep_index = carve<int16_t>(p, g->onep_index.size());
  g->d_basis_prim = carve<int16_t>(p, g->basis_prim.size());
  g->d_ycoef = carve<double>(p, g->ycoef.size());
  g->d_gsrc = carve<int32_t>(p, g->gsrc.size());
  auto put = [](void* d, const void* s, size_t n) { return n ? hipMemcpy(d, s, n, hipMemcpyHostToDevice) : hipSuccess; };
  ACE_HIP(put(g->d_st_ab, g->st_ab.data(), g->st_ab.size() * sizeof(int2)));
  ACE_HIP(put(g->d_st_k, g->st_k.data(), g->st_k.size() * 4));
  ACE_HIP(put(g->d_cl_ab, g->cl_ab.data(), g->cl_ab.size() * sizeof(int2)));
  ACE_HIP(put(g->d_cl_k, g->cl_k.data(), g->cl_k.size() * 4));
  ACE_HIP(put(g->d_leaf_k, g->leaf_k.data(), g->leaf_k.size() * 4));
  ACE_HIP(put(g->d_nv_idx, g->nv_idx.data(), g->nv_idx.size() * 2));
  ACE_HIP(put(g->d_nv_kmap, g->nv_kmap.data(), g->nv_kmap.size() * 4));
  ACE_HIP(put(g->d_nv_slice, g->nv_slice.data(), g->nv_slice.size() * sizeof(int4)));
  ACE_HIP(put(g->d_onep, g->onep.data(), g->onep.size() * sizeof(OnepInfo)));
  ACE_HIP(put(g->d_onep_index, g->onep_index.data(), g->onep_index.size() * 2));
  ACE_HIP(put(g->d_basis_prim, g->basis_prim.data(), g->basis_prim.size() * 2));
  ACE_HIP(put(g->d_ycoef, g->ycoef.data(), g->ycoef.size() * 8));
  ACE_HIP(put(g->d_gsrc, g->gsrc.data(), g->gsrc.size() * 4));

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
  ACE_HIP(hipFuncSetAttribute((const void*)basis_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  ACE_HIP(hipFuncSetAttribute((const void*)basis_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  ACE_HIP(hipFuncSetAttribute((const void*)grad_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  ACE_HIP(hipFuncSetAttribute((const void*)grad_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  ACE_HIP(hipFuncSetAttribute((const void*)planar_grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  ACE_HIP(hipFuncSetAttribute((const void*)planar_basis_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, maxl));
  {
    const ace_status fs = upload_forest(g);
    if (fs != ACE_OK) return fs;
  }
  g->on_device = true;
  return ACE_OK;
}

bool valid_graph(const ace_graph* g) { return g != nullptr; }

ace_status need_device(const ace_graph* g) {
  if (!g) return fail(ACE_ERR_INVALID_ARG, "graph is NULL");
  if (!g->on_device) return fail(ACE_ERR_INVALID_ARG, "graph was built with ACE_BUILD_HOST_ONLY");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != g->device)
    return fail(ACE_ERR_INVALID_ARG, "graph belongs to another HIP device than the current one");
  return ACE_OK;
}

// workspace layout for n_env environments
struct Workspace {
  int32_t* status = nullptr;   // ACE_FLAG_CHECK: result of the offsets' validation (first bytes)
  double2* A = nullptr;
  double2* Abar = nullptr;
  double2* arena_x = nullptr;
  double2* arena_ab = nullptr;
  double* cs = nullptr;   // coefficients in forest-schedule order
  size_t bytes = 0;
};

int arena_blocks(int64_t n_env) { return (int)std::max<int64_t>(1, std::min<int64_t>(n_env, kArenaBlocks)); }

enum class Sched { Layered, Forest, Remat };

bool use_forest(const ace_graph* g, bool grad) {
  const ace_graph::Forest& F = g->fo[0];
  return F.ok && (grad ? F.grad_lds : F.fwd_lds);
}

// The folded forest schedule serves A with the conjugate symmetry when it
// fits; it never holds more resident slots than the unfolded one.
bool use_folded_forest(const ace_graph* g, bool grad) {
  const ace_graph::Forest& F = g->fo[1];
  return F.ok && (grad ? F.grad_lds : F.fwd_lds);
}

// The kernel that evaluates the DAG: the requested schedule when it is
// available, else the forest, else remat, else layer by layer.
Sched pick_schedule(const ace_graph* g, bool grad, uint32_t flags) {
  if (flags & ACE_FLAG_LAYERED) return Sched::Layered;
  const bool f = use_forest(g, grad);
  const bool r = g->remat_ok && g->remat_lds;
  switch (g->opts.schedule) {
    case ACE_SCHEDULE_FOREST:
      if (f) return Sched::Forest;
      break;
    case ACE_SCHEDULE_REMAT:
      if (r) return Sched::Remat;
      break;
    case ACE_SCHEDULE_LAYERED:
      return Sched::Layered;
    default:
      break;
  }
  if (f) return Sched::Forest;
  if (r) return Sched::Remat;
  return Sched::Layered;
}

Workspace plan_workspace(const ace_graph* g, int64_t n_env, uint32_t flags, char* base) {
  Workspace w;
  size_t off = 0;
  auto take = [&](size_t n) {
    char* r = base ? base + off : nullptr;
    off += align_up(n);
    return reinterpret_cast<double2*>(r);
  };
  const size_t per_env = (size_t)g->P1 * sizeof(double2);
  if (flags & ACE_FLAG_CHECK) w.status = reinterpret_cast<int32_t*>(take(sizeof(int32_t)));
  w.A = take((size_t)n_env * per_env);
  w.Abar = take((size_t)n_env * per_env);
  const bool layered = pick_schedule(g, true, flags) == Sched::Layered || pick_schedule(g, false, flags) == Sched::Layered;
  const size_t arena = (size_t)arena_blocks(n_env) * g->slots * sizeof(double2);
  if (layered && (!g->fwd_xl || !g->grad_xl)) w.arena_x = take(arena);
  if (layered && !g->grad_al) w.arena_ab = take(arena);
  size_t ncs = 0;
  for (const auto& F : g->fo)
    if (F.ok) ncs = std::max(ncs, F.kmap.size() * (F.fold ? 2 : 1));
  if (g->remat_ok)
    for (const auto& R : g->rm) ncs = std::max(ncs, R.kmap.size() * (R.fold ? 2 : 1));
  ncs = std::max(ncs, g->nv_kmap.size());
  if (ncs) w.cs = reinterpret_cast<double*>(take(ncs * sizeof(double)));
  w.bytes = off;
  return w;
}

// ACE_FLAG_CHECK: validate the offsets on the device, ahead of the launches
// that read them (which then read no environment if they are invalid); the
// result stays in the workspace for ace_check_offsets_result.  Capture safe.
ace_status launch_check(const int32_t* offsets, int64_t n_env, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(check_offsets_kernel, dim3(1), dim3(1024), 0, s, offsets, n_env, status);
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

int64_t grid_for(int64_t n_env) { return std::max<int64_t>(1, std::min<int64_t>(n_env, (int64_t)1 << 30)); }

// The coefficients of a DAG launch in its schedule order: a separate launch.
ace_status launch_prep(const CoefPrep& c, hipStream_t s) {
  const int64_t nk = c.mode == CoefPrep::kFold ? c.fold.n : c.mode == CoefPrep::kPlain ? c.plain.n : 0;
  if (nk == 0) return ACE_OK;
  const int pgrid = (int)std::max<int64_t>(1, std::min<int64_t>((nk + 255) / 256, 1024));
  if (c.mode == CoefPrep::kFold)
    hipLaunchKernelGGL(prep_fold_kernel, dim3(pgrid), dim3(256), 0, s, c.fold);
  else
    hipLaunchKernelGGL(prep_kernel, dim3(pgrid), dim3(256), 0, s, c.plain);
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

// The preparation of coefficients for a schedule with the given kmap (and
// kbar when folded) into the workspace.
CoefPrep coef_prep(const double* coeffs, const Workspace& w, const int32_t* kmap, const int32_t* kbar, int64_t nk,
                   bool fold) {
  CoefPrep c{};
  if (fold) {
    c.mode = CoefPrep::kFold;
    c.fold.kmap = kmap;
    c.fold.kbar = kbar;
    c.fold.coeffs = coeffs;
    c.fold.cs = reinterpret_cast<double2*>(w.cs);
    c.fold.n = nk;
  } else {
    c.mode = CoefPrep::kPlain;
    c.plain.kmap = kmap;
    c.plain.coeffs = coeffs;
    c.plain.cs = w.cs;
    c.plain.n = nk;
  }
  return c;
}

// Whether two preparations write the same coefficients (same schedule map,
// same coefficients, same output).
bool same_prep(const CoefPrep& a, const CoefPrep& b) {
  if (a.mode != b.mode) return false;
  if (a.mode == CoefPrep::kFold)
    return a.fold.kmap == b.fold.kmap && a.fold.kbar == b.fold.kbar && a.fold.coeffs == b.fold.coeffs &&
           a.fold.cs == b.fold.cs && a.fold.n == b.fold.n;
  if (a.mode == CoefPrep::kPlain)
    return a.plain.kmap == b.plain.kmap && a.plain.coeffs == b.plain.coeffs && a.plain.cs == b.plain.cs &&
           a.plain.n == b.plain.n;
  return true;
}

// prep (may be NULL): a DAG launch's coefficient preparation, done on the
// basis kernel's grid (O(3)) or launched before the planar basis kernel.
ace_status launch_basis(const ace_graph* g, int64_t n_env, const int32_t* offsets, const double* pos, double2* A,
                        hipStream_t s, const CoefPrep* prep, const int32_t* gate = nullptr) {
  if (g->h.spec.group != 0) {
    if (prep) {
      const ace_status st = launch_prep(*prep, s);
      if (st != ACE_OK) return st;
    }
    BasisArgs a{};
    a.n_env = n_env;
    a.offsets = offsets;
    a.pos = pos;
    a.A = A;
    a.onep = g->d_onep;
    a.P1 = g->P1;
    a.n_max = planar_n(g->h);
    a.l_max = planar_m(g->h);
    a.r_cut = g->h.spec.r_cut;
    a.group = g->h.spec.group;
    a.pos_stride = 3;
    a.gate = gate;
    const size_t lds = (size_t)g->P1 * 16 + (size_t)kPlanarChunk * (((a.n_max + 1) + 2 * (a.l_max + 1)) | 1) * 8;
    if (lds > g->max_lds) return fail(ACE_ERR_UNSUPPORTED, "one-particle basis too large for the basis kernel");
    hipLaunchKernelGGL(planar_basis_kernel, dim3((unsigned)grid_for(n_env)), dim3(kBasisThreads), lds, s, a);
    ACE_HIP(hipGetLastError());
    return ACE_OK;
  }
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
  a.group = 0;
  a.k_max = g->h.spec.k_max;
  a.pos_stride = a.k_max > 0 ? 4 : 3;
  a.prim = g->d_basis_prim;
  a.n_prim = (int)g->basis_prim.size();
  a.gate = gate;
  if (prep) a.prep = *prep;
  const int NY = (a.l_max + 1) * (a.l_max + 2) / 2;
  const int chunk = kBasisThreads / (a.l_max + 1);
  const size_t lds = (size_t)g->P1 * 16 + (size_t)chunk * (((a.n_max + 1) + (a.k_max + 1) + 2 * NY) | 1) * 8;
  if (lds > g->max_lds) return fail(ACE_ERR_UNSUPPORTED, "one-particle basis too large for the basis kernel");
  if (a.k_max > 0)
    hipLaunchKernelGGL(basis_kernel<true>, dim3((unsigned)grid_for(n_env)), dim3(kBasisThreads), lds, s, a);
  else
    hipLaunchKernelGGL(basis_kernel<false>, dim3((unsigned)grid_for(n_env)), dim3(kBasisThreads), lds, s, a);
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

CoefPrep forest_prep(const ace_graph* g, const double* coeffs, const Workspace& w, bool fold) {
  const ace_graph::Forest& F = g->fo[fold ? 1 : 0];
  return coef_prep(coeffs, w, F.d_kmap, F.d_kbar, (int64_t)F.kmap.size(), fold);
}

// done (may be NULL): a preparation already on the stream; this launch
// prepares its coefficients itself unless that is the one it needs
ace_status launch_forest(const ace_graph* g, const double* coeffs, int64_t n_env, const double2* A, double2* phi,
                         double2* Abar, const Workspace& w, hipStream_t s, bool fold, const CoefPrep* done) {
  const ace_graph::Forest& F = g->fo[fold ? 1 : 0];
  const CoefPrep need = forest_prep(g, coeffs, w, fold);
  if (!done || !same_prep(*done, need)) {
    const ace_status st = launch_prep(need, s);
    if (st != ACE_OK) return st;
  }
  ForestArgs a{};
  a.n_env = n_env;
  a.A = A;
  a.phi = phi;
  a.Abar = Abar;
  a.cs = w.cs;
  a.nu2_ab = F.d_nu2_ab;
  a.mr_slice = F.d_mr_slice;
  a.mr_row = F.d_mr_row;
  a.me_col = F.d_me_col;
  a.tr_slice = F.d_tr_slice;
  a.it_ab = F.d_it_ab;
  a.ch_s = F.d_ch_s;
  a.ch_g = F.has_gc ? F.d_ch_g : nullptr;
  a.gc_s = F.d_gc_s;
  a.cs_leaf = F.cs_leaf;
  a.cs_me = F.cs_me;
  a.cs_it = F.cs_it;
  a.cs_ch = F.cs_ch;
  a.cs_gc = F.cs_gc;
  a.cs_hot = F.cs_hot;
  a.n_me = (int)F.me_col.size();
  a.n_ch = (int)F.ch_s.size();
  a.n_cs = (int)F.kmap.size();
  a.n_items = F.n_items;
  for (int w = 0; w <= kMaxForestWaves; ++w) {
    a.mr_wave[w] = F.mr_wave[w];
    a.tr_wave[w] = F.tr_wave[w];
  }
  a.hot = make_int4(F.hot_slot[0], F.hot_slot[1], F.hot_slot[2], F.hot_slot[3]);
  a.P1 = g->P1;
  a.N2 = F.N2;
  a.nslot = F.nslot;
  a.n_mslices = F.n_mslices;
  a.n_tslices = F.n_tslices;
  a.fw_ck = F.d_fw_ck;
  a.n_fwck = (int)F.fw_ck.size();
  a.fw_ent = F.d_fw_ent;
  const bool grad = Abar != nullptr;
  // two environments per block where their values fit in LDS
  int ne = g->opts.env_per_block;
  bool full = grad && forest_lds_bytes(F, g->P1, true, true, ne) <= g->max_lds;
  if (ne > 1 && forest_lds_bytes(F, g->P1, grad, full, ne) > g->max_lds) {
    ne = 1;
    full = grad && F.full;
  }
  const size_t lds = forest_lds_bytes(F, g->P1, grad, full, ne);
  const int64_t blocks = (n_env + ne - 1) / ne;
  const dim3 grid((unsigned)grid_for(blocks)), block((unsigned)forest_threads(g));
  const ForestKernel k = forest_variant(ne, fold, full ? 2 : grad ? 1 : 0, F.has_gc);
  hipLaunchKernelGGL(k, grid, block, lds, s, a);
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

CoefPrep remat_prep(const ace_graph* g, const double* coeffs, const Workspace& w, bool grad, bool fold) {
  const ace_graph::Remat& R = g->rm[(fold ? 2 : 0) + (grad ? 1 : 0)];
  return coef_prep(coeffs, w, R.d_kmap, R.d_kbar, (int64_t)R.kmap.size(), fold);
}

ace_status launch_remat(const ace_graph* g, const double* coeffs, int64_t n_env, const double2* A, double2* phi,
                        double2* Abar, const Workspace& w, hipStream_t s, bool fold, const CoefPrep* done) {
  const bool grad = Abar != nullptr;
  const int which = (fold ? 2 : 0) + (grad ? 1 : 0);
  const ace_graph::Remat& R = g->rm[which];
  const CoefPrep need = remat_prep(g, coeffs, w, grad, fold);
  if (!done || !same_prep(*done, need)) {
    const ace_status st = launch_prep(need, s);
    if (st != ACE_OK) return st;
  }
  RematArgs a{};
  a.n_env = n_env;
  a.A = A;
  a.phi = phi;
  a.Abar = Abar;
  a.cs = w.cs;
  a.slice = R.d_slice;
  a.row_lo = R.d_rlo;
  a.row_hi = R.d_rhi;
  a.oth_lo = R.d_olo;
  a.oth_hi = R.d_ohi;
  a.cs_leaf = R.cs_leaf;
  a.cs_ent = R.cs_ent;
  a.P1 = g->P1;
  a.n_slices = R.nslices;
  a.pairs = R.d_pairs;
  a.n_pairs = (int)R.pairs.size();
  a.n_ent = (int)R.olo.size();
  a.hot = make_int4(R.hot[0], R.hot[1], R.hot[2], R.hot[3]);
  const int ne = remat_env_per_block(g, which);
  const size_t lds = remat_lds_bytes(g, which, ne);
  const dim3 grid((unsigned)grid_for((n_env + ne - 1) / ne)), block((unsigned)g->opts.block_threads);
  const bool big = g->opts.block_threads > kRematBlock / 2;
#define ACE_REMAT_LAUNCH(G_, F_, N_, B_) hipLaunchKernelGGL((remat_kernel<G_, F_, N_, B_>), grid, block, lds, s, a)
  switch (which + 4 * (ne - 1) + 8 * (big ? 1 : 0)) {
    case 0: ACE_REMAT_LAUNCH(false, false, 1, false); break;
    case 1: ACE_REMAT_LAUNCH(true, false, 1, false); break;
    case 2: ACE_REMAT_LAUNCH(false, true, 1, false); break;
    case 3: ACE_REMAT_LAUNCH(true, true, 1, false); break;
    case 4: ACE_REMAT_LAUNCH(false, false, 2, false); break;
    case 5: ACE_REMAT_LAUNCH(true, false, 2, false); break;
    case 6: ACE_REMAT_LAUNCH(false, true, 2, false); break;
    case 7: ACE_REMAT_LAUNCH(true, true, 2, false); break;
    case 8: ACE_REMAT_LAUNCH(false, false, 1, true); break;
    case 9: ACE_REMAT_LAUNCH(true, false, 1, true); break;
    case 10: ACE_REMAT_LAUNCH(false, true, 1, true); break;
    case 11: ACE_REMAT_LAUNCH(true, true, 1, true); break;
    case 12: ACE_REMAT_LAUNCH(false, false, 2, true); break;
    case 13: ACE_REMAT_LAUNCH(true, false, 2, true); break;
    case 14: ACE_REMAT_LAUNCH(false, true, 2, true); break;
    default: ACE_REMAT_LAUNCH(true, true, 2, true); break;
  }
#undef ACE_REMAT_LAUNCH
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

// conj_ok: A satisfies A_{n,l,-m} = (-1)^m conj(A_{n,l,m}) (it comes from
// the basis kernel), so schedules with folded conjugate pairs may be used.
// The coefficient preparation launch_dag needs for these arguments (mode
// kNone for the layered schedule, which reads c directly).
CoefPrep dag_prep(const ace_graph* g, const double* coeffs, const Workspace& w, bool grad, uint32_t flags,
                  bool conj_ok) {
  switch (pick_schedule(g, grad, flags)) {
    case Sched::Forest:
      return forest_prep(g, coeffs, w, conj_ok && !(flags & ACE_FLAG_UNFOLDED) && use_folded_forest(g, grad));
    case Sched::Remat:
      return remat_prep(g, coeffs, w, grad, conj_ok && !(flags & ACE_FLAG_UNFOLDED));
    default:
      return CoefPrep{};
  }
}

// done (may be NULL): a coefficient preparation already on the stream
// (dag_prep's for the same arguments, normally)
ace_status launch_dag(const ace_graph* g, const double* coeffs, int64_t n_env, const double2* A, double2* phi,
                      double2* Abar, const Workspace& w, hipStream_t s, uint32_t flags, bool conj_ok,
                      const CoefPrep* done = nullptr) {
  switch (pick_schedule(g, Abar != nullptr, flags)) {
    case Sched::Forest:
      return launch_forest(g, coeffs, n_env, A, phi, Abar, w, s,
                           conj_ok && !(flags & ACE_FLAG_UNFOLDED) && use_folded_forest(g, Abar != nullptr), done);
    case Sched::Remat:
      return launch_remat(g, coeffs, n_env, A, phi, Abar, w, s, conj_ok && !(flags & ACE_FLAG_UNFOLDED), done);
    default:
      break;
  }
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
                        double2* Abar, const Workspace& w, hipStream_t s) {
  CoefPrep prep{};
  prep.mode = CoefPrep::kPlain;
  prep.plain.kmap = g->d_nv_kmap;
  prep.plain.coeffs = coeffs;
  prep.plain.cs = w.cs;
  prep.plain.n = (int64_t)g->nv_kmap.size();
  ace_status st = launch_prep(prep, s);
  if (st != ACE_OK) return st;
  NaiveArgs a{};
  a.n_env = n_env;
  a.A = A;
  a.phi = phi;
  a.Abar = Abar;
  a.cs = w.cs;
  a.slice = g->d_nv_slice;
  a.idx = g->d_nv_idx;
  a.n_slices = (int)g->nv_slice.size();
  a.P1 = g->P1;
  const size_t lds = (size_t)(2 * (g->P1 + 1) + kNaiveBlock / 64) * sizeof(double2);
  if (lds > g->max_lds) return fail(ACE_ERR_UNSUPPORTED, "one-particle basis too large for the naive kernel");
  const dim3 grid((unsigned)grid_for(n_env)), block(kNaiveBlock);
  if (Abar)
    hipLaunchKernelGGL(naive_kernel<true>, grid, block, lds, s, a);
  else
    hipLaunchKernelGGL(naive_kernel<false>, grid, block, lds, s, a);
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

ace_status launch_grad(const ace_graph* g, int64_t n_env, const int32_t* offsets, const double* pos,
                       const double2* Abar, double* grad, hipStream_t s, const int32_t* gate = nullptr) {
  if (g->h.spec.group != 0) {
    GradArgs a{};
    a.n_env = n_env;
    a.offsets = offsets;
    a.pos = pos;
    a.Abar = Abar;
    a.grad = grad;
    a.P1 = g->P1;
    a.n_max = planar_n(g->h);
    a.l_max = planar_m(g->h);
    a.r_cut = g->h.spec.r_cut;
    a.group = g->h.spec.group;
    a.pidx = g->d_onep_index;
    a.pos_stride = 3;
    a.gate = gate;
    const int NR = g->h.spec.group == 2 ? a.n_max : 0;
    const size_t lds = (size_t)g->P1 * sizeof(double2) +
                       (size_t)kPlanarChunk * (((kPlanarNbr + 2 * (NR + 1) + 2 * (a.l_max + 1)) | 1) + 2) * 8;
    if (lds > g->max_lds) return fail(ACE_ERR_UNSUPPORTED, "one-particle basis too large for the gradient kernel");
    hipLaunchKernelGGL(planar_grad_kernel, dim3((unsigned)grid_for(n_env)), dim3(kGradThreads), lds, s, a);
    ACE_HIP(hipGetLastError());
    return ACE_OK;
  }
  GradArgs a{};
  a.n_env = n_env;
  a.offsets = offsets;
  a.pos = pos;
  a.Abar = Abar;
  a.grad = grad;
  a.onep_index = g->d_onep_index;
  a.gsrc = reinterpret_cast<const int2*>(g->d_gsrc);
  a.ycoef = g->d_ycoef;
  a.P1 = g->P1;
  a.n_max = g->h.spec.n_max;
  a.l_max = g->h.spec.l_max;
  a.r_cut = g->h.spec.r_cut;
  a.group = 0;
  a.k_max = g->h.spec.k_max;
  a.pos_stride = a.k_max > 0 ? 4 : 3;
  a.gate = gate;
  const int NY = (a.l_max + 1) * (a.l_max + 2) / 2;
  const size_t lds = (g->gsrc.size() / 2) * sizeof(double2) + (size_t)((3 * NY + 1) & ~1) * 8 +
                     (size_t)kGradChunk * (grad_nbr_doubles(a.n_max) + 3) * 8;
  if (lds > g->max_lds) return fail(ACE_ERR_UNSUPPORTED, "one-particle basis too large for the gradient kernel");
  a.nb = g->grad_nb;
  if (a.k_max > 0)
    hipLaunchKernelGGL(grad_kernel<true>, dim3((unsigned)grid_for(n_env)), dim3(kGradWave), lds, s, a);
  else
    hipLaunchKernelGGL(grad_kernel<false>, dim3((unsigned)grid_for(n_env)), dim3(kGradWave), lds, s, a);
  ACE_HIP(hipGetLastError());
  return ACE_OK;
}

ace_status common_eval_checks(const ace_graph* g, const double* coeffs, int64_t n_env, const void* workspace,
                              size_t ws_bytes, uint32_t flags, size_t* need) {
  ace_status st = need_device(g);
  if (st != ACE_OK) return st;
  if (n_env < 0) return fail(ACE_ERR_INVALID_ARG, "n_env must be >= 0");
  if (n_env > ((int64_t)1 << 30)) return fail(ACE_ERR_INVALID_ARG, "n_env too large");
  if (flags & ~(ACE_FLAG_NAIVE | ACE_FLAG_CHECK | ACE_FLAG_LAYERED | ACE_FLAG_UNFOLDED | ACE_FLAG_CONJ_SYMMETRIC))
    return fail(ACE_ERR_INVALID_ARG, "unknown flag bits");
  if (n_env == 0) return ACE_OK;
  if (!coeffs) return fail(ACE_ERR_INVALID_ARG, "coeffs is NULL");
  *need = plan_workspace(g, n_env, flags, nullptr).bytes;
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
    bs.degree_p = spec->degree_p == 0 ? 1 : spec->degree_p;
    bs.k_max = spec->k_max;
    bs.r_cut = spec->r_cut;
    build_graph(bs, g->h);
    make_schedule(g);
    make_forest(g, 0);
    make_forest(g, 1);
    make_remat(g);
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
  if (g->fmem) (void)hipFree(g->fmem);
  if (g->rmem) (void)hipFree(g->rmem);
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

ace_status ace_graph_export_feature(const ace_graph* g, int32_t* k) {
  if (!g || !k) return fail(ACE_ERR_INVALID_ARG, "graph and k must be non-NULL");
  std::memcpy(k, g->h.on_k.data(), g->h.on_k.size() * 4);
  return ACE_OK;
}

ace_status ace_graph_export_k(const ace_graph* g, int32_t* k_tuples) {
  if (!g || !k_tuples) return fail(ACE_ERR_INVALID_ARG, "graph and k_tuples must be non-NULL");
  std::memcpy(k_tuples, g->h.k_flat.data(), g->h.k_flat.size() * 4);
  return ACE_OK;
}

ace_status ace_workspace_size(const ace_graph* g, int64_t n_env, int64_t n_nbr, uint32_t flags, size_t* bytes) {
  (void)n_nbr;
  if (!g || !bytes) return fail(ACE_ERR_INVALID_ARG, "graph and bytes must be non-NULL");
  if (n_env < 0) return fail(ACE_ERR_INVALID_ARG, "n_env must be >= 0");
  if (!g->on_device) return fail(ACE_ERR_INVALID_ARG, "graph was built with ACE_BUILD_HOST_ONLY");
  *bytes = plan_workspace(g, n_env, flags, nullptr).bytes;
  return ACE_OK;
}

ace_status ace_basis(const ace_graph* g, int64_t n_env, const int32_t* offsets, const double* pos, double* A,
                     void* stream) {
  ace_status st = need_device(g);
  if (st != ACE_OK) return st;
  if (n_env < 0) return fail(ACE_ERR_INVALID_ARG, "n_env must be >= 0");
  if (n_env == 0) return ACE_OK;
  if (!offsets || !pos || !A) return fail(ACE_ERR_INVALID_ARG, "offsets, pos and A must be non-NULL");
  return launch_basis(g, n_env, offsets, pos, reinterpret_cast<double2*>(A), (hipStream_t)stream, nullptr);
}

ace_status ace_contract(const ace_graph* g, const double* coeffs, int64_t n_env, const double* A, double* phi,
                        double* Abar, void* workspace, size_t ws_bytes, uint32_t flags, void* stream) {
  size_t need = 0;
  ace_status st = common_eval_checks(g, coeffs, n_env, workspace, ws_bytes, flags, &need);
  if (st != ACE_OK || n_env == 0) return st;
  if (!A || !phi) return fail(ACE_ERR_INVALID_ARG, "A and phi must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  const Workspace w = plan_workspace(g, n_env, flags, static_cast<char*>(workspace));
  if (flags & ACE_FLAG_NAIVE)
    return launch_naive(g, coeffs, n_env, reinterpret_cast<const double2*>(A), reinterpret_cast<double2*>(phi),
                        reinterpret_cast<double2*>(Abar), w, s);
  return launch_dag(g, coeffs, n_env, reinterpret_cast<const double2*>(A), reinterpret_cast<double2*>(phi),
                    reinterpret_cast<double2*>(Abar), w, s, flags, (flags & ACE_FLAG_CONJ_SYMMETRIC) != 0);
}

ace_status ace_eval(const ace_graph* g, const double* coeffs, int64_t n_env, const int32_t* offsets,
                    const double* pos, double* phi, void* workspace, size_t ws_bytes, uint32_t flags, void* stream) {
  size_t need = 0;
  ace_status st = common_eval_checks(g, coeffs, n_env, workspace, ws_bytes, flags, &need);
  if (st != ACE_OK || n_env == 0) return st;
  if (!offsets || !pos || !phi) return fail(ACE_ERR_INVALID_ARG, "offsets, pos and phi must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  const Workspace w = plan_workspace(g, n_env, flags, static_cast<char*>(workspace));
  if (flags & ACE_FLAG_CHECK) {
    st = launch_check(offsets, n_env, w.status, s);
    if (st != ACE_OK) return st;
  }
  if (flags & ACE_FLAG_NAIVE) {
    st = launch_basis(g, n_env, offsets, pos, w.A, s, nullptr, w.status);
    if (st != ACE_OK) return st;
    return launch_naive(g, coeffs, n_env, w.A, reinterpret_cast<double2*>(phi), nullptr, w, s);
  }
  // the DAG launch's coefficients are prepared on the basis kernel's grid
  const CoefPrep prep = dag_prep(g, coeffs, w, false, flags, true);
  st = launch_basis(g, n_env, offsets, pos, w.A, s, &prep, w.status);
  if (st != ACE_OK) return st;
  return launch_dag(g, coeffs, n_env, w.A, reinterpret_cast<double2*>(phi), nullptr, w, s, flags, true, &prep);
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
  const Workspace w = plan_workspace(g, n_env, flags, static_cast<char*>(workspace));
  if (flags & ACE_FLAG_CHECK) {
    st = launch_check(offsets, n_env, w.status, s);
    if (st != ACE_OK) return st;
  }
  if (flags & ACE_FLAG_NAIVE) {
    st = launch_basis(g, n_env, offsets, pos, w.A, s, nullptr, w.status);
    if (st != ACE_OK) return st;
    st = launch_naive(g, coeffs, n_env, w.A, reinterpret_cast<double2*>(phi), w.Abar, w, s);
  } else {
    // the DAG launch's coefficients are prepared on the basis kernel's grid
    const CoefPrep prep = dag_prep(g, coeffs, w, true, flags, true);
    st = launch_basis(g, n_env, offsets, pos, w.A, s, &prep, w.status);
    if (st != ACE_OK) return st;
    st = launch_dag(g, coeffs, n_env, w.A, reinterpret_cast<double2*>(phi), w.Abar, w, s, flags, true, &prep);
  }
  if (st != ACE_OK) return st;
  return launch_grad(g, n_env, offsets, pos, w.Abar, grad, s, w.status);
}

ace_status ace_check_offsets_result(const void* workspace) {
  if (!workspace) return fail(ACE_ERR_INVALID_ARG, "workspace is NULL");
  int32_t v = -1;
  ACE_HIP(hipMemcpy(&v, workspace, sizeof(v), hipMemcpyDeviceToHost));
  switch (v) {
    case 0: return ACE_OK;
    case 1: return fail(ACE_ERR_INVALID_ARG, "offsets[0] must be 0 (device-side validation)");
    case 2: return fail(ACE_ERR_INVALID_ARG, "offsets must be non-decreasing (device-side validation)");
    default: return fail(ACE_ERR_INVALID_ARG, "no offsets validation result in this workspace");
  }
}

ace_status ace_eval_grad_noalloc(const ace_graph* g, const double* coeffs, int64_t n_env, const int32_t* offsets,
                                 const double* pos, double* phi, double* grad, uint32_t flags, void* stream) {
  ace_status st = need_device(g);
  if (st != ACE_OK) return st;
  if (n_env < 0) return fail(ACE_ERR_INVALID_ARG, "n_env must be >= 0");
  if (n_env > ((int64_t)1 << 30)) return fail(ACE_ERR_INVALID_ARG, "n_env too large");
  if (flags & ACE_FLAG_CHECK)
    return fail(ACE_ERR_INVALID_ARG, "ace_eval_grad_noalloc does not take ACE_FLAG_CHECK");
  if (flags & ~(ACE_FLAG_NAIVE | ACE_FLAG_LAYERED | ACE_FLAG_UNFOLDED))
    return fail(ACE_ERR_INVALID_ARG, "unknown flag bits");
  if (n_env == 0) return ACE_OK;
  const size_t need = plan_workspace(g, n_env, flags, nullptr).bytes;
  if (need > kNoallocScratchBytes)
    return fail(ACE_ERR_INVALID_ARG, "ace_eval_grad_noalloc: " + std::to_string(n_env) + " environments need " +
                                         std::to_string(need) + " bytes of workspace, more than its fixed " +
                                         std::to_string(kNoallocScratchBytes) + "; split the batch");
  void* ws = nullptr;
  st = scratch_address(g->device, &ws);
  if (st != ACE_OK) return st;
  return ace_eval_grad(g, coeffs, n_env, offsets, pos, phi, grad, ws, kNoallocScratchBytes, flags, stream);
}

ace_status ace_graph_get_schedule(const ace_graph* g, ace_schedule_opts* o) {
  if (!g || !o) return fail(ACE_ERR_INVALID_ARG, "graph and opts must be non-NULL");
  std::memset(o, 0, sizeof(*o));
  o->row_chunk = g->opts.row_chunk;
  o->tree_chunk = g->opts.tree_chunk;
  o->hot_columns = g->opts.hot_columns;
  o->bank_schedule = g->opts.bank_schedule;
  o->block_threads = g->opts.block_threads;
  o->schedule = g->opts.schedule;
  o->term_chunk = g->opts.term_chunk;
  o->pair_slots = g->opts.pair_slots;
  o->env_per_block = g->opts.env_per_block;
  return ACE_OK;
}

ace_status ace_graph_set_schedule(ace_graph* g, const ace_schedule_opts* o) {
  if (!g || !o) return fail(ACE_ERR_INVALID_ARG, "graph and opts must be non-NULL");
  if (o->row_chunk < 4 || o->row_chunk > 256 || o->tree_chunk < 1 || o->tree_chunk > 256 || o->hot_columns < 0 ||
      o->hot_columns > 4 || (o->bank_schedule != 0 && o->bank_schedule != 1) || o->block_threads < 64 ||
      o->block_threads > 1024 || o->block_threads % 64 != 0 || o->schedule < ACE_SCHEDULE_AUTO ||
      o->schedule > ACE_SCHEDULE_LAYERED || o->term_chunk < 1 || o->term_chunk > 256 ||
      o->pair_slots < -1 || o->pair_slots > 8192 || o->env_per_block < 1 || o->env_per_block > 2)
    return fail(ACE_ERR_INVALID_ARG, "schedule option out of range");
  if (g->on_device) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != g->device)
      return fail(ACE_ERR_INVALID_ARG, "graph belongs to another HIP device than the current one");
  }
  // The current schedules (host layouts and the device copies their pointers
  // name) stay intact until the new ones are built and uploaded; any failure
  // puts them back together with every option.
  const ScheduleOpts old = g->opts;
  ace_graph::Forest old_fo[2];
  ace_graph::Remat old_rm[4];
  for (int i = 0; i < 2; ++i) {
    old_fo[i] = std::move(g->fo[i]);
    g->fo[i] = ace_graph::Forest{};
  }
  for (int i = 0; i < 4; ++i) {
    old_rm[i] = std::move(g->rm[i]);
    g->rm[i] = ace_graph::Remat{};
  }
  const bool old_remat_ok = g->remat_ok, old_remat_lds = g->remat_lds;
  std::string old_remat_why = g->remat_why;
  void* old_fmem = g->fmem;
  void* old_rmem = g->rmem;
  auto restore = [&]() {
    if (g->fmem != old_fmem && g->fmem) (void)hipFree(g->fmem);
    if (g->rmem != old_rmem && g->rmem) (void)hipFree(g->rmem);
    g->fmem = old_fmem;
    g->rmem = old_rmem;
    g->opts = old;
    for (int i = 0; i < 2; ++i) g->fo[i] = std::move(old_fo[i]);
    for (int i = 0; i < 4; ++i) g->rm[i] = std::move(old_rm[i]);
    g->remat_ok = old_remat_ok;
    g->remat_lds = old_remat_lds;
    g->remat_why = old_remat_why;
  };
  g->opts.row_chunk = o->row_chunk;
  g->opts.tree_chunk = o->tree_chunk;
  g->opts.hot_columns = o->hot_columns;
  g->opts.bank_schedule = o->bank_schedule;
  g->opts.block_threads = o->block_threads;
  g->opts.schedule = o->schedule;
  g->opts.term_chunk = o->term_chunk;
  g->opts.pair_slots = o->pair_slots;
  g->opts.env_per_block = o->env_per_block;
  try {
    make_forest(g, 0);
    make_forest(g, 1);
    make_remat(g);
  } catch (const std::bad_alloc&) {
    restore();
    return fail(ACE_ERR_OUT_OF_MEMORY, "host allocation failed while rebuilding the schedule");
  }
  if (o->schedule == ACE_SCHEDULE_FOREST && !g->fo[0].ok) {
    const std::string why = g->fo[0].why;
    restore();
    return fail(ACE_ERR_UNSUPPORTED, "no forest schedule for this graph: " + why);
  }
  if (o->schedule == ACE_SCHEDULE_REMAT && !g->remat_ok) {
    const std::string why = g->remat_why;
    restore();
    return fail(ACE_ERR_UNSUPPORTED, "no remat schedule for this graph: " + why);
  }
  if (g->on_device) {
    // upload_forest allocates fresh device blocks; the old ones are freed
    // only once the new ones are in place
    g->fmem = nullptr;
    g->rmem = nullptr;
    const ace_status st = upload_forest(g);
    if (st != ACE_OK) {
      const std::string msg = ace_last_error();
      restore();
      return fail(st, msg);
    }
    if (old_fmem) (void)hipFree(old_fmem);
    if (old_rmem) (void)hipFree(old_rmem);
  }
  return ACE_OK;
}

ace_status ace_debug_schedule(const ace_graph* g, int32_t* kind, int64_t* info) {
  if (!g || !kind) return fail(ACE_ERR_INVALID_ARG, "graph and kind must be non-NULL");
  Sched sc;
  if (g->on_device) {
    sc = pick_schedule(g, true, 0);
  } else {
    // host-only graph: what a device with 160 KiB of LDS per block would pick
    const size_t lds = 160 * 1024;
    const bool f = g->fo[0].ok && forest_lds_bytes(g->fo[0], g->P1, true, false) <= lds;
    const bool r = g->remat_ok && remat_lds_bytes(g, 1) <= lds && remat_lds_bytes(g, 3) <= lds;
    const int want = g->opts.schedule;
    if (want == ACE_SCHEDULE_LAYERED) sc = Sched::Layered;
    else if (want == ACE_SCHEDULE_REMAT && r) sc = Sched::Remat;
    else if (f) sc = Sched::Forest;
    else if (r) sc = Sched::Remat;
    else sc = Sched::Layered;
  }
  *kind = sc == Sched::Forest ? 1 : sc == Sched::Remat ? 2 : 0;
  if (sc != Sched::Forest) g_error = g->fo[0].ok ? "forest schedule not selected" : g->fo[0].why;
  if (info) {
    for (int i = 0; i < 16; ++i) info[i] = 0;
    if (sc == Sched::Remat) {
      const ace_graph::Remat& R = g->rm[1];
      info[0] = g->P1 + 1 + (int64_t)R.pairs.size();
      info[1] = R.nslices;
      info[2] = (int64_t)R.olo.size();
      int64_t real = 0;
      for (size_t i = R.cs_ent; i < R.kmap.size(); ++i) real += R.kmap[i] != -1;
      info[3] = real;
      info[4] = R.nitems;
      info[5] = g->rm[0].nslices;
      info[6] = (int64_t)g->rm[0].olo.size();
      int64_t real0 = 0;
      for (size_t i = g->rm[0].cs_ent; i < g->rm[0].kmap.size(); ++i) real0 += g->rm[0].kmap[i] != -1;
      info[7] = real0;
      for (int k = 0; k < 4; ++k) info[8 + k] = R.hot[k];
      info[12] = (int64_t)R.pairs.size();
      // mean LDS cycles of the 16-byte factor reads of the entries per
      // quarter-wave (x1000): the LDS serves a quarter in max(2, m) cycles,
      // m the most distinct slots in one bank group (slot mod 16)
      int64_t cost = 0, nq = 0;
      for (const int4& sl : R.slice) {
        const int sig = sl.w >> 8;
        for (int j = 0; j < sl.z; ++j)
          for (int u = 0; u < sig; ++u)
            for (int q = 0; q < 4; ++q) {
              int slots[16];
              for (int i = 0; i < 16; ++i) {
                const size_t e = (size_t)sl.y + (size_t)j * 64 + 16 * q + i;
                const uint64_t w = u < 4 ? R.olo[e] : R.ohi[e];
                slots[i] = (int)(((w >> (16 * (u & 3))) & 0xffffu) >> 4);
              }
              int mx = 0;
              for (int b = 0; b < 16; ++b) {
                int d = 0;
                for (int i = 0; i < 16; ++i) {
                  if ((slots[i] & 15) != b) continue;
                  bool first = true;
                  for (int k = 0; k < i; ++k) first &= slots[k] != slots[i];
                  d += first;
                }
                mx = std::max(mx, d);
              }
              cost += std::max(2, mx);   // LDS cycles of the quarter: two slots per bank group are free
              ++nq;
            }
      }
      info[13] = nq ? (1000 * cost) / nq : 0;
      int64_t real3 = 0;
      for (size_t i = g->rm[3].cs_ent; i < g->rm[3].kmap.size(); ++i) real3 += g->rm[3].kmap[i] != -1;
      info[14] = real3;
      // mean LDS bank load of the row pushes (8-byte atomics into the Re or
      // Im plane, served a quarter-wave at a time over 16 bank pairs, slot
      // mod 16): per push instruction and quarter, the most lanes on one
      // bank pair (x1000)
      const int nh = std::min(g->opts.hot_columns, g->opts.env_per_block > 1 ? 2 : 4);
      int64_t pcost = 0, npq = 0;
      for (const int4& sl : R.slice) {
        const int nb = sl.w & 0xff;
        for (int i = 0; i < nb; ++i)
          for (int q = 0; q < 4; ++q) {
            int cnt[16] = {0};
            bool any = false;
            for (int l = 16 * q; l < 16 * q + 16; ++l) {
              const size_t it = (size_t)sl.x + l;
              const uint64_t w = i < 4 ? R.rlo[it] : R.rhi[it];
              const int s = (int)(((w >> (16 * (i & 3))) & 0xffffu) >> 4);
              const int s0 = (int)((R.rlo[it] & 0xffffu) >> 4);
              bool hot = s == g->P1 || s0 == g->P1;   // constant slot, or a padding lane (no pushes)
              for (int k = 0; k < nh; ++k) hot |= s == R.hot[k];
              if (hot) continue;
              cnt[s & 15] += 1;
              any = true;
            }
            if (!any) continue;
            pcost += *std::max_element(cnt, cnt + 16);
            ++npq;
          }
      }
      info[15] = npq ? (1000 * pcost) / npq : 0;
    }
    if (sc == Sched::Forest) {
      const ace_graph::Forest& F = g->fo[0];
      info[0] = F.nslot;
      info[1] = F.n_tslices;
      info[2] = (int64_t)F.ch_s.size();
      int64_t realc = 0;
      for (uint16_t v : F.ch_s) realc += v != (uint16_t)g->P1;
      info[3] = realc;
      info[4] = F.n_mslices;
      info[5] = (int64_t)F.me_col.size();
      int64_t reale = 0;
      for (int32_t k : std::vector<int32_t>(F.kmap.begin() + F.cs_me, F.kmap.begin() + F.cs_nu2)) reale += k != -1;
      info[6] = reale;
      info[7] = (int64_t)F.gc_s.size();
      for (int h = 0; h < 4; ++h) info[8 + h] = F.hot_slot[h];
      info[12] = F.full ? 1 : 0;
      // LDS bank cost of the 16-byte gathers: sum over gathers and quarters of
      // the largest number of lanes sharing a bank group (ideal: 1 each)
      auto cost = [](const uint16_t* sl) {   // distinct slots per bank group (same slot: broadcast)
        int64_t c = 0;
        for (int q = 0; q < 4; ++q) {
          int mx = 0;
          for (int b = 0; b < 16; ++b) {
            int d = 0;
            for (int i = 0; i < 16; ++i) {
              const int v = sl[16 * q + i];
              if ((v & 15) != b) continue;
              bool first = true;
              for (int k = 0; k < i; ++k) first &= sl[16 * q + k] != v;
              d += first;
            }
            mx = std::max(mx, d);
          }
          c += mx;
        }
        return c;
      };
      int64_t cm = 0, ct = 0, nm = 0, nt = 0;
      for (size_t pos = 0; pos + 64 <= F.me_col.size(); pos += 64, ++nm) cm += cost(&F.me_col[pos]);
      for (size_t pos = 0; pos + 64 <= F.ch_s.size(); pos += 64, ++nt) ct += cost(&F.ch_s[pos]);
      info[13] = nm ? (1000 * cm) / (4 * nm) : 0;   // mean per quarter, x1000
      info[14] = nt ? (1000 * ct) / (4 * nt) : 0;
      int64_t realf = 0;   // real tree children and pair entries of the folded schedule
      const ace_graph::Forest& F1 = g->fo[1];
      if (F1.ok) {
        for (uint16_t v : F1.ch_s) realf += v != (uint16_t)g->P1;
        for (int i = F1.cs_me; i < F1.cs_nu2; ++i) realf += F1.kmap[i] != -1;
      }
      info[15] = realf;
    }
  }
  return ACE_OK;
}

ace_status ace_debug_forest_eval(const ace_graph* g, const double* coeffs, int64_t n_env, const double* A,
                                 double* phi, double* Abar, int32_t folded) {
  if (!g || !coeffs || !A || !phi || !Abar || n_env < 0) return fail(ACE_ERR_INVALID_ARG, "NULL argument");
  const int which = folded ? 1 : 0;
  if (!g->fo[which].ok) return fail(ACE_ERR_UNSUPPORTED, "no forest schedule: " + g->fo[which].why);
  std::vector<double> phi2(2), ab2(2 * (size_t)g->P1);
  for (int64_t e = 0; e < n_env; ++e) {
    // both adjoint modes; they must agree
    if (!forest_emulate(g, which, coeffs, A + 2 * e * g->P1, phi + 2 * e, Abar + 2 * e * g->P1, true) ||
        !forest_emulate(g, which, coeffs, A + 2 * e * g->P1, phi2.data(), ab2.data(), false))
      return fail(ACE_ERR_INTERNAL, "forest schedule index out of range");
    double num = 0.0, den = 0.0;
    for (int i = 0; i < 2 * g->P1; ++i) {
      const double d = ab2[i] - Abar[2 * e * g->P1 + i];
      num += d * d;
      den += ab2[i] * ab2[i];
    }
    if (num > 1e-24 * (den + 1e-300)) return fail(ACE_ERR_INTERNAL, "forest adjoint modes disagree");
  }
  return ACE_OK;
}

ace_status ace_debug_remat_eval(const ace_graph* g, const double* coeffs, int64_t n_env, const double* A,
                                double* phi, double* Abar, int32_t folded) {
  if (!g || !coeffs || !A || !phi || !Abar || n_env < 0) return fail(ACE_ERR_INVALID_ARG, "NULL argument");
  if (!g->remat_ok) return fail(ACE_ERR_UNSUPPORTED, "no remat schedule: " + g->remat_why);
  const int base = folded ? 2 : 0;
  double phi1[2];
  for (int64_t e = 0; e < n_env; ++e) {
    // both schedules; their phi must agree
    if (!remat_emulate(g, base + 1, coeffs, A + 2 * e * g->P1, phi + 2 * e, Abar + 2 * e * g->P1) ||
        !remat_emulate(g, base, coeffs, A + 2 * e * g->P1, phi1, nullptr))
      return fail(ACE_ERR_INTERNAL, "remat schedule index out of range");
    const double d = std::hypot(phi1[0] - phi[2 * e], phi1[1] - phi[2 * e + 1]);
    if (d > 1e-10 * (std::hypot(phi1[0], phi1[1]) + 1e-300)) return fail(ACE_ERR_INTERNAL, "remat schedules disagree");
  }
  return ACE_OK;
}

}  // extern "C"
