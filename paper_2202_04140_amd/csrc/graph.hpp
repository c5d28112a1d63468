// Host-side construction of the recursive-evaluation DAG.
//
// Sec. 2.6: a tuple k = [k1, k2] (multiset union) is evaluated as the
// product A_k = A_k1 * A_k2; tuples with no invariant split need auxiliary,
// non-invariant nodes with zero coefficient.  Algorithm 1 (Sec. 3.2) and
// Algorithm 2 (Sec. 3.3) insert every tuple of K in increasing correlation
// order.  This file holds the index sets, the two insertion heuristics and
// the layering; the GPU schedules are derived from it in schedule.cpp.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ace {

struct BuildSpec {
  int group = 0;       // 0 = O(3), 1 = torus
  int nu_max = 0;
  int degree_max = 0;
  int n_max = 0;
  int l_max = 0;
  int algorithm = 1;
  int alg_n = 1;
  int degree_p = 1;    // 1, 2, or -1 for p = infinity (Sec. 2.5)
  int k_max = 0;       // O(3): degree of the invariant-feature polynomials T_k (Sec. 5.4)
  double r_cut = 5.0;
};

// Open-addressing map from a sorted tuple of one-particle indices to a
// node id.  Keys live in the graph's flat tuple array; the table stores ids.
class TupleIndex {
 public:
  void init(int width, size_t expected);
  // returns node id or -1
  int32_t find(const int32_t* key, int len, const std::vector<int32_t>& flat,
               const std::vector<int8_t>& lens) const;
  void insert(int32_t id, const int32_t* key, int len, const std::vector<int32_t>& flat,
              const std::vector<int8_t>& lens);

 private:
  static uint64_t hash(const int32_t* key, int len);
  void grow(const std::vector<int32_t>& flat, const std::vector<int8_t>& lens);
  int width_ = 0;
  size_t count_ = 0;
  std::vector<int32_t> slots_;
};

struct HostGraph {
  BuildSpec spec;
  int width = 0;  // = nu_max, row length of the flat tuple arrays

  // one-particle list in canonical order (n+l, l, m) (torus: (|m|, m))
  int P1 = 0;
  std::vector<int32_t> on_n, on_l, on_m, on_k, on_deg;

  // K in canonical order: by length, then lexicographic
  int64_t nK = 0;
  int64_t nK_by_order[9] = {0};
  std::vector<int32_t> k_flat;  // [nK][width], -1 padded
  std::vector<int8_t> k_len;

  // nodes in insertion order
  std::vector<int32_t> node_flat;  // [V][width], -1 padded
  std::vector<int8_t> node_len;
  std::vector<int32_t> par;        // [V][2], -1 for one-particle nodes
  std::vector<int64_t> k_to_node;  // [nK]
  std::vector<int32_t> node_k;     // [V] index into K or -1 (auxiliary)

  // derived
  std::vector<int32_t> layer;   // [V]
  std::vector<int32_t> nchild;  // [V] number of child edges (a square counts twice)
  int depth = 0;

  int64_t n_nodes() const { return (int64_t)node_len.size(); }
};

// Builds everything above.  Throws std::invalid_argument / std::bad_alloc.
void build_graph(const BuildSpec& spec, HostGraph& g);

}  // namespace ace
