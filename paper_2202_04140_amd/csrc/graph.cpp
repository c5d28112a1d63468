// Host-side DAG construction: index sets (Sec. 2.3-2.5, Sec. 3), the
// node-insertion heuristics of Algorithm 1 (Sec. 3.2) and Algorithm 2
// (Sec. 3.3), and the layering of the resulting graph (Sec. 2.6).
//
// Choices the paper leaves open, fixed here:
//  * canonical one-particle order (n+l, l, m) for O(3) and (|m|, m) for the
//    torus; tuples are non-decreasing index lists, so the last element has
//    the largest degree;
//  * K is inserted by length, then lexicographically;
//  * the split search tries the smaller part's size s = floor(nu/2) down to
//    1, position combinations in lexicographic order, and takes the first
//    split whose two parts are already nodes; parents are stored as
//    (sub-multiset, complement);
//  * Algorithm 1 splits off the last element, Algorithm 2 the last
//    min(n, nu-1) elements (a maximal-degree sub-tuple for p = 1); the node
//    is then inserted by searching again;
//  * one-particle nodes get ids 0..P1-1 before any tuple; ids follow
//    insertion order.
#include "graph.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

namespace ace {

// ---------------------------------------------------------------------------
// TupleIndex
// ---------------------------------------------------------------------------
uint64_t TupleIndex::hash(const int32_t* key, int len) {
  uint64_t h = 0x9E3779B97F4A7C15ull ^ (uint64_t)len;
  for (int i = 0; i < len; ++i) {
    h ^= (uint64_t)(uint32_t)key[i] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 31;
  }
  return h;
}

void TupleIndex::init(int width, size_t expected) {
  width_ = width;
  size_t cap = 1024;
  while (cap < expected * 2) cap <<= 1;
  slots_.assign(cap, -1);
  count_ = 0;
}

static inline bool same_key(const int32_t* a, int la, const int32_t* b, int lb) {
  if (la != lb) return false;
  for (int i = 0; i < la; ++i)
    if (a[i] != b[i]) return false;
  return true;
}

int32_t TupleIndex::find(const int32_t* key, int len, const std::vector<int32_t>& flat,
                         const std::vector<int8_t>& lens) const {
  const size_t mask = slots_.size() - 1;
  size_t p = hash(key, len) & mask;
  while (true) {
    int32_t id = slots_[p];
    if (id < 0) return -1;
    if (same_key(key, len, &flat[(size_t)id * width_], lens[id])) return id;
    p = (p + 1) & mask;
  }
}

void TupleIndex::grow(const std::vector<int32_t>& flat, const std::vector<int8_t>& lens) {
  std::vector<int32_t> old;
  old.swap(slots_);
  slots_.assign(old.size() * 2, -1);
  const size_t mask = slots_.size() - 1;
  for (int32_t id : old) {
    if (id < 0) continue;
    size_t p = hash(&flat[(size_t)id * width_], lens[id]) & mask;
    while (slots_[p] >= 0) p = (p + 1) & mask;
    slots_[p] = id;
  }
}

void TupleIndex::insert(int32_t id, const int32_t* key, int len, const std::vector<int32_t>& flat,
                        const std::vector<int8_t>& lens) {
  if ((count_ + 1) * 2 > slots_.size()) grow(flat, lens);
  const size_t mask = slots_.size() - 1;
  size_t p = hash(key, len) & mask;
  while (slots_[p] >= 0) p = (p + 1) & mask;
  slots_[p] = id;
  ++count_;
}

// ---------------------------------------------------------------------------
// builder
// ---------------------------------------------------------------------------
namespace {

struct Builder {
  HostGraph& g;
  TupleIndex index;
  explicit Builder(HostGraph& gr) : g(gr) {}

  int32_t find(const int32_t* k, int len) const { return index.find(k, len, g.node_flat, g.node_len); }

  int32_t add(const int32_t* k, int len, int32_t a, int32_t b) {
    const int32_t id = (int32_t)g.node_len.size();
    if (id == INT32_MAX) throw std::length_error("too many DAG nodes");
    for (int i = 0; i < g.width; ++i) g.node_flat.push_back(i < len ? k[i] : -1);
    g.node_len.push_back((int8_t)len);
    g.par.push_back(a);
    g.par.push_back(b);
    index.insert(id, k, len, g.node_flat, g.node_len);
    return id;
  }

  // "for all decompositions k = [k1, k2]: if k1, k2 in G: add k" -- the
  // search order is the one fixed in the header comment.
  bool try_split(const int32_t* k, int len) {
    int32_t k1[8], k2[8];
    int pos[8];
    for (int s = len / 2; s >= 1; --s) {
      // first combination 0..s-1
      for (int i = 0; i < s; ++i) pos[i] = i;
      while (true) {
        // build k1 (positions) and k2 (complement), both sorted since k is
        int a = 0, b = 0, q = 0;
        for (int i = 0; i < len; ++i) {
          if (q < s && pos[q] == i) {
            k1[a++] = k[i];
            ++q;
          } else {
            k2[b++] = k[i];
          }
        }
        const int32_t i1 = find(k1, s);
        if (i1 >= 0) {
          const int32_t i2 = find(k2, len - s);
          if (i2 >= 0) {
            add(k, len, i1, i2);
            return true;
          }
        }
        // next combination in lexicographic order
        int i = s - 1;
        while (i >= 0 && pos[i] == len - s + i) --i;
        if (i < 0) break;
        ++pos[i];
        for (int j = i + 1; j < s; ++j) pos[j] = pos[j - 1] + 1;
      }
    }
    return false;
  }

  // Algorithm 1 (Sec. 3.2)
  void insert_alg1(const int32_t* k, int len) {
    if (find(k, len) >= 0) return;
    if (try_split(k, len)) return;
    // split off the maximal-degree one-particle factor (the last element);
    // the one-particle node is always present, insert the rest, then retry
    insert_alg1(k, len - 1);
    insert_alg1(k, len);
  }

  // Algorithm 2 (Sec. 3.3) with parameter n
  void insert_alg2(const int32_t* k, int len, int n) {
    if (find(k, len) >= 0) return;
    if (try_split(k, len)) return;
    const int s = std::min(n, len - 1);
    insert_alg1(k + (len - s), s);  // maximal-degree sub-tuple, by Algorithm 1
    insert_alg2(k, len - s, n);
    insert_alg2(k, len, n);
  }
};

// one-particle list (Sec. 2.4 / 2.3), canonical order
void make_onebody(HostGraph& g) {
  const BuildSpec& s = g.spec;
  struct T {
    int n, l, m, deg, k = 0;
  };
  std::vector<T> v;
  if (s.group == 0) {
    // with an invariant feature (Sec. 5.4) the degree is n + l + k; the order
    // (deg, l, k, m) keeps the 2l+1 functions of one (n, l, k) consecutive
    for (int n = 0; n <= s.n_max; ++n)
      for (int l = 0; l <= s.l_max; ++l)
        for (int k = 0; k <= s.k_max; ++k)
          if (n + l + k <= s.degree_max)
            for (int m = -l; m <= l; ++m) v.push_back({n, l, m, n + l + k, k});
    std::stable_sort(v.begin(), v.end(), [](const T& a, const T& b) {
      if (a.deg != b.deg) return a.deg < b.deg;
      if (a.l != b.l) return a.l < b.l;
      if (a.k != b.k) return a.k < b.k;
      return a.m < b.m;
    });
  } else if (s.group == 2) {
    // SO(2) (Sec. 2.2): (n, m), n <= n_max, |m| <= m_max (= l_max), degree n + |m|;
    // the l field holds |m| so that (n, l, -m) is the conjugate function
    for (int n = 0; n <= s.n_max; ++n)
      for (int m = -s.l_max; m <= s.l_max; ++m) {
        const int am = m < 0 ? -m : m;
        if (n + am <= s.degree_max) v.push_back({n, am, m, n + am});
      }
    std::stable_sort(v.begin(), v.end(), [](const T& a, const T& b) {
      if (a.deg != b.deg) return a.deg < b.deg;
      if (a.l != b.l) return a.l < b.l;
      return a.m < b.m;
    });
  } else {
    for (int m = -s.degree_max; m <= s.degree_max; ++m) v.push_back({0, 0, m, m < 0 ? -m : m});
    std::stable_sort(v.begin(), v.end(), [](const T& a, const T& b) {
      if (a.deg != b.deg) return a.deg < b.deg;
      return a.m < b.m;
    });
  }
  g.P1 = (int)v.size();
  for (const T& t : v) {
    g.on_n.push_back(t.n);
    g.on_l.push_back(t.l);
    g.on_m.push_back(t.m);
    g.on_k.push_back(t.k);
    g.on_deg.push_back(t.deg);
  }
}

// K_G^p(nu, D) for nu = 1..nu_max (Sec. 2.5, Sec. 3), depth-first in
// lexicographic order.  `budget` is what is left of D (p = 1), of D^2
// (p = 2, sum of squared degrees) or D itself (p = infinity).
void enumerate_k(HostGraph& g) {
  const int P = g.P1;
  const int D = g.spec.degree_max;
  const int p = g.spec.degree_p;
  const bool check_l = g.spec.group == 0;
  int32_t cur[8];
  for (int nu = 1; nu <= g.spec.nu_max; ++nu) {
    struct Rec {
      static void go(HostGraph& g, int32_t* cur, int depth, int nu, int start, int budget, int msum, int lsum,
                     int P, bool check_l, int p, int D) {
        if (depth == nu) {
          if (msum != 0) return;
          if (check_l && (lsum & 1)) return;
          for (int i = 0; i < g.width; ++i) g.k_flat.push_back(i < nu ? cur[i] : -1);
          g.k_len.push_back((int8_t)nu);
          return;
        }
        const int left = nu - depth;
        for (int i = start; i < P; ++i) {
          const int d = g.on_deg[i];
          // later elements have degree >= d
          const int cost = p == 2 ? d * d : (p == 1 ? d : 0);
          if (p == -1 ? d > D : cost * left > budget) break;
          const int ms = msum + g.on_m[i];
          // |m| <= deg for every later element: bound how far the m-sum can still move
          const int rest = budget - cost;
          int reach;
          if (p == 1)
            reach = rest;
          else if (p == 2)
            reach = (int)std::floor(std::sqrt((double)(left - 1) * (double)rest) + 1e-9);
          else
            reach = (left - 1) * D;
          if ((ms < 0 ? -ms : ms) > reach) continue;
          cur[depth] = i;
          go(g, cur, depth + 1, nu, i, rest, ms, lsum + g.on_l[i], P, check_l, p, D);
        }
      }
    };
    const size_t before = g.k_len.size();
    Rec::go(g, cur, 0, nu, 0, p == 2 ? D * D : D, 0, 0, P, check_l, p, D);
    g.nK_by_order[nu] = (int64_t)(g.k_len.size() - before);
  }
  g.nK = (int64_t)g.k_len.size();
}

}  // namespace

void build_graph(const BuildSpec& spec, HostGraph& g) {
  if (spec.group < 0 || spec.group > 2) throw std::invalid_argument("group must be 0 (O3), 1 (torus) or 2 (SO2)");
  if (spec.nu_max < 1 || spec.nu_max > 8) throw std::invalid_argument("nu_max must be in 1..8");
  if (spec.degree_max < 0 || spec.degree_max > 64) throw std::invalid_argument("degree_max must be in 0..64");
  if (spec.group == 0 || spec.group == 2) {
    if (spec.n_max < 0 || spec.n_max > 64) throw std::invalid_argument("n_max must be in 0..64");
    if (spec.l_max < 0 || spec.l_max > (spec.group == 0 ? 16 : 64))
      throw std::invalid_argument(spec.group == 0 ? "l_max must be in 0..16" : "m_max (l_max) must be in 0..64");
  }
  if (spec.algorithm != 1 && spec.algorithm != 2) throw std::invalid_argument("algorithm must be 1 or 2");
  if (spec.algorithm == 2 && spec.alg_n < 1) throw std::invalid_argument("alg_n must be >= 1");
  if (spec.k_max < 0 || spec.k_max > 16) throw std::invalid_argument("k_max must be in 0..16");
  if (spec.k_max > 0 && spec.group != 0) throw std::invalid_argument("invariant features need the O(3) group");
  if (spec.degree_p != 1 && spec.degree_p != 2 && spec.degree_p != -1)
    throw std::invalid_argument("degree_p must be 1, 2 or -1 (infinity)");
  if (!(spec.r_cut > 0.0)) throw std::invalid_argument("r_cut must be > 0");

  g = HostGraph();
  g.spec = spec;
  g.width = spec.nu_max;
  make_onebody(g);
  enumerate_k(g);

  Builder b(g);
  b.index.init(g.width, (size_t)(g.nK + g.P1) + (size_t)(g.nK / 8));
  g.node_flat.reserve((size_t)(g.nK + g.P1) * g.width * 11 / 10);
  g.node_len.reserve((size_t)(g.nK + g.P1) * 11 / 10);
  g.par.reserve((size_t)(g.nK + g.P1) * 2 * 11 / 10);

  // Sec. 2.6: first the one-particle nodes
  for (int i = 0; i < g.P1; ++i) {
    int32_t k = i;
    b.add(&k, 1, -1, -1);
  }
  // then every tuple of K in increasing correlation order
  for (int64_t q = 0; q < g.nK; ++q) {
    const int32_t* k = &g.k_flat[(size_t)q * g.width];
    const int len = g.k_len[q];
    if (spec.algorithm == 1)
      b.insert_alg1(k, len);
    else
      b.insert_alg2(k, len, spec.alg_n);
  }

  const int64_t V = g.n_nodes();
  g.k_to_node.resize(g.nK);
  g.node_k.assign(V, -1);
  for (int64_t q = 0; q < g.nK; ++q) {
    const int32_t id = b.find(&g.k_flat[(size_t)q * g.width], g.k_len[q]);
    if (id < 0) throw std::logic_error("tuple of K missing from the graph");
    g.k_to_node[q] = id;
    g.node_k[id] = (int32_t)q;
  }

  g.layer.assign(V, 0);
  g.nchild.assign(V, 0);
  g.depth = 0;
  for (int64_t v = 0; v < V; ++v) {
    const int32_t a = g.par[2 * v], c = g.par[2 * v + 1];
    if (a < 0) continue;
    g.layer[v] = 1 + std::max(g.layer[a], g.layer[c]);
    g.depth = std::max(g.depth, g.layer[v]);
    g.nchild[a] += 1;
    g.nchild[c] += 1;
  }
}

}  // namespace ace
