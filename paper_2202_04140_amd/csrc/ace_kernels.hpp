// Device-side argument blocks shared by the kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ace {

constexpr int kMaxLayers = 16;

// One-particle basis (Sec. 2.4): per one-particle index i its n, the offset
// of (l, |m|) in the per-neighbour Y table, and the signs mapping
// Y_l^{|m|} to Y_l^{m} (Y_l^{-m} = (-1)^m conj(Y_l^m)).
struct OnepInfo {
  int16_t n;
  int16_t yoff;   // (l*(l+1))/2 + |m|
  int8_t sre;     // +1 / -1 applied to Re Y_l^{|m|}
  int8_t sim;     // +1 / -1 applied to Im Y_l^{|m|}
  int8_t l;
  int8_t am;      // |m|
  int8_t k;       // feature degree (Sec. 5.4), 0 without a feature
  int16_t neg;    // O(3), m > 0: index of the (n, l, -m, k) function; else -1
};

struct PrepFoldArgs {
  const int32_t* kmap;   // k >= 0: c_k;  -1: 0;  k <= -2: doubled c_{-2-k}
  const int32_t* kbar;   // conjugate partner of k, or -1 if k is self-conjugate
  const double* coeffs;  // [|K|]
  double2* cs;           // output (Re weight, Im weight)
  int64_t n;
};

struct PrepArgs {
  const int32_t* kmap;   // k >= 0: c_k;  -1: 0;  k <= -2: 2 c_{-2-k}
  const double* coeffs;  // [|K|]
  double* cs;            // output
  int64_t n;
};

// The coefficient preparation of one DAG launch, done by another kernel
// of the same step (the basis kernel): none, plain or folded.
struct CoefPrep {
  enum { kNone = 0, kPlain = 1, kFold = 2 };
  int mode;
  PrepArgs plain;
  PrepFoldArgs fold;
};

struct BasisArgs {
  int64_t n_env;
  const int32_t* offsets;
  const double* pos;
  double2* A;            // [n_env][P1]
  const OnepInfo* onep;  // [P1]
  const double* ycoef;   // [3][(L+1)*(L+2)/2]: A, B, start (start only at l = m)
  int P1, n_max, l_max;
  double r_cut;
  int group;             // 0 O(3); planar: 1 torus, 2 SO(2)
  int k_max;             // O(3) feature degree; positions then carry mu as a fourth column
  int pos_stride;        // doubles per position: 3, or 4 with a feature
  const int16_t* prim;   // O(3): [n_prim] indices of the functions with m >= 0
  int n_prim;
  CoefPrep prep;         // O(3): the next DAG launch's coefficients, prepared on this grid
  const int32_t* gate;   // device status of the offsets' validation (ACE_FLAG_CHECK): nonzero
                         // means invalid and no environment is read; nullptr: no validation
};

// Planar one-particle functions (torus, SO(2)): phi_i = R_n(r) e^{i s m theta}
// with E_{|m|} = ((x + i y)/r)^{|m|}: phi_i = R_n (Re E, sim Im E) where
// OnepInfo.sim = s * sign(m) (s = +1 torus, -1 SO(2)); R_n = 1 for the torus.

// Forward / adjoint DAG schedule.  Value slots: one-particle nodes
// 0..P1-1, stored product nodes (nodes with a child) P1..P1+S-1 in layer
// order.  Childless product nodes have no slot.
struct DagArgs {
  int64_t n_env;
  const double2* A;      // [n_env][P1]
  double2* phi;          // [n_env]
  double2* Abar;         // [n_env][P1] or nullptr (forward only)
  const double* coeffs;  // [|K|]
  const int2* st_ab;     // [S] parent slots of stored nodes
  const int32_t* st_k;   // [S] K index or -1
  const int2* cl_ab;     // [T] parent slots of childless nodes
  const int32_t* cl_k;   // [T] K index
  const int32_t* leaf_k; // [P1] K index or -1
  double2* arena_x;      // [gridDim][slots] when the value arena is not in LDS
  double2* arena_ab;     // [gridDim][slots] when the adjoint arena is not in LDS
  int P1, S, slots, depth;
  int st_off[kMaxLayers + 2];  // stored nodes of layer L: [st_off[L], st_off[L+1])
  int cl_off[kMaxLayers + 2];
};

// Naive schedule: the tuples of each length in slices of 64 lanes, each lane
// taking kNaiveChunk consecutive tuples (in K order); a slice's factor
// indices are stored [step][factor][lane] and its coefficients [step][lane],
// padding tuples hold the constant-one slot P1 and a zero coefficient.
struct NaiveArgs {
  int64_t n_env;
  const double2* A;
  double2* phi;
  double2* Abar;
  const double* cs;       // prepared coefficients in slice order
  const int4* slice;      // [n_slices] {first index, first coefficient, length nu, steps}
  const int16_t* idx;     // factor indices
  int n_slices;
  int P1;
};

struct GradArgs {
  int64_t n_env;
  const int32_t* offsets;
  const double* pos;
  const double2* Abar;       // [n_env][P1]
  double* grad;              // [n_nbr][3]
  const int16_t* onep_index; // [(n_max+1)][(l_max+1)][(2 l_max+1)] -> i or -1
  const int2* gsrc;          // [(l_max+1)(l_max+2)/2][nb]: at (l(l+1)/2+m) nb + n (k_max+1) + k, m >= 0, the
                             // functions (n, l, +-m, k): (i of +m or -1, i of -m as i (m even) or -2-i (m odd), or -1)
  const double* ycoef;
  int P1, n_max, l_max;
  double r_cut;
  int group;                 // 0 O(3); planar: 1 torus, 2 SO(2)
  const int16_t* pidx;       // planar: [(n_max+1)][(2 m_max+1)] -> i or -1 (m_max = l_max)
  int k_max;                 // O(3) feature degree
  int pos_stride;            // doubles per position: 3, or 4 with a feature
  int nb;                    // O(3): entries per (l, m) of the staged Abar (odd, >= (n_max+1)(k_max+1))
  const int32_t* gate;       // as BasisArgs::gate
};

}  // namespace ace

namespace ace {

constexpr int kMaxForestWaves = 8;   // forest kernel: waves per block at most (512 threads)
constexpr int kForwardChunk = 8;     // forest, full-adjoint mode: forwarding entries per chunk

// Forest schedule (see forest_kernel).  Value slots: one-particle nodes
// 0..P1-1, a constant-zero slot P1, then the order-2 nodes P1+1..P1+N2.
// Slot numbers fit in 16 bits.  Coefficients are read from `cs`, the
// per-call copy of c in schedule order, at the given offsets.
struct ForestArgs {
  int64_t n_env;
  const double2* A;          // [n_env][P1]
  double2* phi;              // [n_env]
  double2* Abar;             // [n_env][P1], or nullptr for the forward pass only
  const double* cs;          // prepared coefficients (double2 pairs for a folded schedule)
  const uint32_t* nu2_ab;    // [N2] parent one-particle slots, a | b << 16
  const int4* mr_slice;      // [n_mslices] {first row, first entry, entries per row, 0}
  const uint16_t* mr_row;    // [64 * n_mslices] row slot of each resident-pair row
  const uint16_t* me_col;    // resident-pair entries, 64-interleaved per slice
  const int4* tr_slice;      // [n_tslices] {first item, first child, children per item, 0}
  const uint32_t* it_ab;     // [64 * n_tslices] root parents, a | b << 16
  const uint16_t* ch_s;      // children, 64-interleaved per slice: resident sibling slot
  const int2* ch_g;          // children: grandchild range [x, y) (nullptr if none exist)
  const uint16_t* gc_s;      // grandchildren: resident sibling slot
  int cs_leaf, cs_me, cs_it, cs_ch, cs_gc, cs_hot;
  int n_me, n_ch, n_cs;      // sizes of me_col, ch_s and cs (in coefficients; byte sizes below 2^31)
  int P1, N2, nslot, n_mslices, n_tslices;
  int n_items;   // 64 * n_tslices
  int4 hot;      // slots of the four hot-sibling columns (P1 = unused)
  // wave w of a block takes pair-row slices [mr_wave[w], mr_wave[w + 1]) and
  // tree slices [tr_wave[w], tr_wave[w + 1]) (balanced on the host)
  int mr_wave[kMaxForestWaves + 1];
  int tr_wave[kMaxForestWaves + 1];
  // full-adjoint mode: abar for every resident slot in LDS, order-2
  // adjoints forwarded at the end: chunk c {one-particle slot i, ...}
  // gathers sum abar_u x_other over its kForwardChunk entries
  // fw_ent[c * kForwardChunk ...] and adds it to abar_i
  const int4* fw_ck;       // [n_fwck]
  int n_fwck;
  const uint32_t* fw_ent;  // [n_fwck * kForwardChunk] order-2 slot | (other parent slot << 16)
};

// Rematerialising schedule (see remat_kernel).  LDS slots: one-particle
// nodes 0..P1-1, a constant-one slot P1 (padding), then n_pairs products of
// two one-particle values.  Factor lists hold the LDS byte offset 16 * slot
// of each factor, 16 bits each, four to a 64-bit word; unused fields hold
// 16 * P1.  Row factors are one-particle slots only.
struct RematArgs {
  int64_t n_env;
  const double2* A;          // [n_env][P1]
  double2* phi;              // [n_env]
  double2* Abar;             // [n_env][P1], or nullptr for the forward pass only
  const double* cs;          // prepared coefficients (double2 pairs for a folded schedule)
  const int4* slice;         // [n_slices] {first item, first entry, entries per item, nrow | nother << 8}
  const uint64_t* row_lo;    // [n_items] row factors 0..3
  const uint64_t* row_hi;    // [n_items] row factors 4..7
  const uint64_t* oth_lo;    // entries, 64-interleaved per slice: factors 0..3 of the other parent
  const uint64_t* oth_hi;    // entries: factors 4..7 (read only when the other parent has more than 4)
  const uint32_t* pairs;     // [n_pairs] one-particle slots a | b << 16 of the pair products
  int cs_leaf, cs_ent;
  int P1, n_slices, n_pairs;
  int n_ent;                 // entry positions (at most 2^26: byte offsets of the entry loads fit in 31 bits)
  int4 hot;                  // one-particle slots whose adjoints are summed in registers (P1 = unused)
};

}  // namespace ace
