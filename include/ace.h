/*
 * ace.h -- C ABI of the MI355X (gfx950) evaluator for symmetry-adapted
 * n-correlations by recursive contraction over a product DAG.
 *
 * Method: Kaliuzhnyi & Ortner, "Optimal Evaluation of Symmetry-Adapted
 * n-Correlations Via Recursive Contraction of Sparse Symmetric Tensors"
 * (arXiv:2202.04140).
 *
 *   phi = sum_{nu=1}^{nu_max} sum_{k in K} c_k prod_{t=1}^{nu} A_{k_t}
 *                                                       (Eq. (1.1), Eq. (2.1))
 *   A_{nlm} = sum_j R_n(|r_j|) Y_l^m(r_j / |r_j|)        (Sec. 2.1, Sec. 2.4)
 *   K = sorted tuples with sum m = 0, sum l even,
 *       sum (n + l) <= D                                  (Sec. 2.4, 2.5, 3)
 *
 * The tuples of K are evaluated through a DAG in which every node of
 * correlation order >= 2 is the product of two earlier nodes, with the
 * auxiliary (non-invariant, zero-coefficient) nodes the sparsity requires,
 * built by the insertion heuristic of Algorithm 1 (Sec. 2.6, Sec. 3.2) or
 * Algorithm 2 (Sec. 3.3).
 *
 * Conventions shared by every entry point
 *   - All floating point is IEEE binary64.  Complex numbers are stored as
 *     interleaved (re, im) pairs of doubles.
 *   - Every function returns an ace_status; ACE_OK is 0.  On failure a
 *     human readable message is available from ace_last_error() (thread
 *     local, valid until the next failing call on the same thread).  No C++
 *     exception crosses this boundary.
 *   - "device" pointers are HIP device allocations on the current device
 *     (the caller allocates and frees them; the library never frees a
 *     caller pointer).  "host" pointers are ordinary process memory.
 *   - Evaluation calls are asynchronous on the given stream (a hipStream_t
 *     passed as void*, NULL = the legacy default stream); results are valid
 *     once the stream has been synchronised.  They allocate no memory: the
 *     caller supplies a device workspace of at least ace_workspace_size()
 *     bytes.  Calls that share a workspace must not overlap in time.
 *   - Radial basis: R_n(r) = T_n(cos(pi r / r_cut)) (Chebyshev polynomials
 *     of the first kind), n = 0..n_max.  Angular basis: complex, orthonormal
 *     spherical harmonics with the Condon-Shortley phase and e^{+i m phi}
 *     azimuthal factor, so Y_l^{-m} = (-1)^m conj(Y_l^m).
 *   - One-particle order (the index i of A_i): triples (n, l, m) sorted by
 *     (n + l, l, m) ascending.  Tuples are non-decreasing lists of such
 *     indices; K is ordered by length, then lexicographically.  The
 *     coefficient array c of every call follows this order of K.
 */
#ifndef ACE_H_
#define ACE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ace_status;

#define ACE_OK                0
#define ACE_ERR_INVALID_ARG   1  /* a NULL pointer, negative size, bad spec ... */
#define ACE_ERR_UNSUPPORTED   2  /* valid request this build does not implement */
#define ACE_ERR_OUT_OF_MEMORY 3  /* host or device allocation failed (graph build) */
#define ACE_ERR_HIP           4  /* a HIP runtime call failed */
#define ACE_ERR_INTERNAL      5  /* internal consistency check failed */

/* symmetry group of the one-particle basis (Sec. 2.2-2.4) */
#define ACE_GROUP_O3    0   /* phi_nlm = R_n Y_l^m, sum m = 0 and sum l even (Sec. 2.4) */
#define ACE_GROUP_TORUS 1   /* phi_m = e^{i m theta}, sum m = 0 (Sec. 2.3)              */
#define ACE_GROUP_SO2   2   /* phi_nm = R_n(r) e^{-i m theta}, sum m = 0 (Sec. 2.2)      */

/* ace_basis_spec.build_flags */
#define ACE_BUILD_HOST_ONLY 1u  /* build the DAG on the host only, no device upload */

/* flags of the evaluation calls */
#define ACE_FLAG_NAIVE 1u  /* evaluate each tuple's product directly (baseline) */
#define ACE_FLAG_CHECK 2u  /* ace_eval / ace_eval_grad: validate the offsets on
                              the device ahead of the launches that read them
                              (offsets[0] = 0, non-decreasing); if invalid those
                              launches read no environment and the outputs are
                              unspecified.  The result stays in the workspace:
                              read it with ace_check_offsets_result once the
                              stream has been synchronised.  No synchronisation
                              in the call: capture safe. */
#define ACE_FLAG_LAYERED 4u /* evaluate the DAG layer by layer even where the
                              forest schedule applies (for testing) */
#define ACE_FLAG_UNFOLDED 8u /* ace_eval / ace_eval_grad: evaluate every tuple of K
                              even where the schedule could fold conjugate pairs
                              (for testing) */
#define ACE_FLAG_CONJ_SYMMETRIC 16u /* ace_contract: the caller guarantees
                              A[e][(n,l,-m)] = (-1)^m conj(A[e][(n,l,m)]), as ace_basis
                              produces, so conjugate pairs of K may be folded (one
                              tuple per pair is evaluated).  Abar then satisfies
                              Re sum_i Abar_i dA_i = d Re(phi) for such dA but is not
                              dphi/dA itself.  ace_eval / ace_eval_grad imply it. */

/*
 * Basis specification (Sec. 2.5, Sec. 3).
 *   group       ACE_GROUP_O3 or ACE_GROUP_TORUS
 *   nu_max      maximal correlation order, 1 <= nu_max <= 8
 *   degree_max  D >= 0: degree cutoff ||k||_p <= D over the element degrees
 *               n_t + l_t (torus: |m_t|); every one-particle function has
 *               n + l <= D
 *   n_max,l_max radial / angular cutoffs: O(3) n <= n_max, l <= l_max <= 16;
 *               SO(2) n <= n_max, |m| <= l_max <= 64; unused for the torus.
 *               Planar groups read positions as (x, y) (the z entry is
 *               ignored), theta = atan2(y, x), r = |(x, y)|.
 *   algorithm   1 = Algorithm 1 (Sec. 3.2), 2 = Algorithm 2 (Sec. 3.3)
 *   alg_n       Algorithm 2's parameter n >= 1 (ignored for algorithm 1)
 *   degree_p    ACE_DEGREE_P1 (total degree, also 0), ACE_DEGREE_P2 (sum of
 *               squared degrees <= D^2) or ACE_DEGREE_PINF (largest degree <= D)
 *   r_cut       radial scale of R_n (> 0)
 *   k_max       O(3) only, 0..16: one invariant feature mu per neighbour
 *               (Sec. 5.4), phi_nlmk = R_n Y_l^m T_k(mu) with Chebyshev T_k,
 *               k <= k_max, degree n + l + k (0: no feature).  With k_max > 0
 *               positions are [n_nbr][4] = (x, y, z, mu), mu in [-1, 1]; the
 *               gradients stay [n_nbr][3].
 */
#define ACE_DEGREE_P1 1
#define ACE_DEGREE_P2 2
#define ACE_DEGREE_PINF (-1)
typedef struct ace_basis_spec {
  int32_t group;
  int32_t nu_max;
  int32_t degree_max;
  int32_t n_max;
  int32_t l_max;
  int32_t algorithm;
  int32_t alg_n;
  int32_t degree_p;
  double r_cut;
  uint32_t build_flags;
  int32_t k_max;
} ace_basis_spec;

/* Graph statistics (Sec. 3.1: K, D/I split is not computed; A = aux). */
typedef struct ace_graph_stats {
  int64_t n_onep;            /* P1: one-particle functions                   */
  int64_t n_k;               /* |K| over all orders                          */
  int64_t n_k_by_order[9];   /* |K_G(nu, D)| for nu = 0..8 (index 0 unused)  */
  int64_t n_nodes;           /* V: all DAG nodes including one-particle ones */
  int64_t n_aux;             /* auxiliary nodes (product, not invariant)     */
  int64_t n_aux_by_order[9];
  int64_t depth;             /* number of product layers                     */
  int64_t n_stored;          /* product nodes with at least one child        */
  int64_t n_childless;       /* product nodes with no child                  */
  int64_t n_leaf_parents;    /* one-particle nodes that have a child         */
  int64_t n_layer[16];       /* nodes per layer (layer 0 = one-particle)     */
  int64_t naive_cmuls;       /* sum over K of (nu - 1)                       */
} ace_graph_stats;

typedef struct ace_graph ace_graph;

/* Message of the last failing call on this thread ("" if none). */
const char* ace_last_error(void);

/* Library version string (static storage). */
const char* ace_version(void);

/*
 * Build the DAG for `spec` on the host (K enumeration, Algorithm 1 or 2,
 * layering, evaluation schedules) and, unless ACE_BUILD_HOST_ONLY is set,
 * upload the schedules to the current HIP device.  Synchronous.  On success
 * *out owns host and device memory until ace_graph_free.  The graph is
 * immutable afterwards and may be shared by concurrent calls on any stream.
 * Errors: ACE_ERR_INVALID_ARG (spec out of range), ACE_ERR_OUT_OF_MEMORY,
 * ACE_ERR_HIP (device upload failed).
 */
ace_status ace_graph_build(const ace_basis_spec* spec, ace_graph** out);

/*
 * Tunable parameters of the evaluation schedule (not of the DAG itself;
 * the node list and every result are unchanged up to rounding order).
 *   row_chunk      resident-pair entries handled per lane item, 4..256
 *   tree_chunk     children of a tree root handled per lane item, 1..256
 *   hot_columns    number of most frequent sibling slots given register
 *                  accumulators instead of per-child atomics, 0..4
 *   bank_schedule  1: order work so that a quarter-wave's LDS gathers hit
 *                  distinct bank groups; 0: plain order
 *   block_threads  threads per block of the DAG kernel, 64..1024, multiple
 *                  of 64 (the forest kernel takes at most 512)
 *   schedule       which DAG kernel evaluates the graph (ACE_SCHEDULE_*):
 *                  AUTO takes the forest schedule when its resident set
 *                  fits in LDS, else the remat schedule, else the layered
 *                  one.  FOREST and REMAT fail with ACE_ERR_UNSUPPORTED in
 *                  ace_graph_set_schedule when the graph has no such
 *                  schedule.
 *   term_chunk     remat schedule: terms sharing a base handled per lane
 *                  item, 1..256
 *   pair_slots     remat schedule: products of two one-particle values
 *                  precomputed in LDS per environment and used as factors,
 *                  0..8192 (the most frequent pairs are taken), or -1: as
 *                  many as fit without lowering the kernel's occupancy
 *   env_per_block  forest and remat schedules: environments one block
 *                  evaluates together, sharing every schedule and
 *                  coefficient load, 1 or 2 (2 falls back to 1 where two
 *                  environments' values do not fit in LDS)
 * hot_columns also sets the number of one-particle slots whose adjoints
 * the remat kernel sums in registers (at most 2 with two environments per
 * block).  The kernels read schedule metadata with 32-bit byte offsets: a
 * remat schedule of more than 2^26 entries, or a forest schedule of more
 * than 2^27 coefficients, is not built (the graph then has no such
 * schedule, and AUTO takes the next one).
 */
#define ACE_SCHEDULE_AUTO 0
#define ACE_SCHEDULE_FOREST 1   /* one-particle and order-2 values resident in LDS */
#define ACE_SCHEDULE_REMAT 2    /* one-particle values resident, parents recomputed */
#define ACE_SCHEDULE_LAYERED 3  /* layer by layer, value arenas in LDS or HBM */

typedef struct ace_schedule_opts {
  int32_t row_chunk;
  int32_t tree_chunk;
  int32_t hot_columns;
  int32_t bank_schedule;
  int32_t block_threads;
  int32_t schedule;
  int32_t term_chunk;
  int32_t pair_slots;
  int32_t env_per_block;
} ace_schedule_opts;

/* Current schedule options of a graph (host). */
ace_status ace_graph_get_schedule(const ace_graph* g, ace_schedule_opts* opts);

/*
 * Rebuild the evaluation schedule with new options and, for a device graph,
 * re-upload it (synchronous; allocates device memory owned by the graph).
 * Must not overlap with evaluation calls on the same graph.
 * ACE_ERR_INVALID_ARG if an option is out of range.
 */
ace_status ace_graph_set_schedule(ace_graph* g, const ace_schedule_opts* opts);

/* Release a graph (NULL is a no-op).  No call using it may be in flight. */
void ace_graph_free(ace_graph* g);

/* Fill *stats (host).  Sec. 3.1 node and auxiliary counts. */
ace_status ace_graph_info(const ace_graph* g, ace_graph_stats* stats);

/*
 * Copy the node list into caller-allocated HOST buffers (any may be NULL):
 *   onep      [P1][3]       int32 (n, l, m) of each one-particle function
 *                           (torus: (0, 0, m))
 *   node_tuple[V][nu_max]   int32 sorted one-particle indices, -1 padded
 *   parents   [V][2]        int32 parent node ids in insertion order
 *                           (Sec. 2.6 k = [k1, k2]); -1 for one-particle nodes
 *   k_to_node [|K|]         int64 node id of every tuple of K
 * Node ids are insertion order (one-particle nodes 0..P1-1 first).
 */
ace_status ace_graph_export(const ace_graph* g, int32_t* onep, int32_t* node_tuple,
                            int32_t* parents, int64_t* k_to_node);

/* Copy the tuples of K into a caller HOST buffer [|K|][nu_max], -1 padded. */
ace_status ace_graph_export_k(const ace_graph* g, int32_t* k_tuples);

/* Feature degree k of every one-particle function (host int32 [P1]; all 0
 * without a feature). */
ace_status ace_graph_export_feature(const ace_graph* g, int32_t* k);

/*
 * Device workspace (bytes) needed by the evaluation calls below for n_env
 * environments and n_nbr neighbour vectors in total, with `flags`.
 */
ace_status ace_workspace_size(const ace_graph* g, int64_t n_env, int64_t n_nbr,
                              uint32_t flags, size_t* bytes);

/*
 * One-particle basis with pooling, Sec. 2.1 Eq. (2.1) and Sec. 2.4:
 *   A[e][i] = sum_{j in env e} R_{n_i}(|r_j|) Y_{l_i}^{m_i}(r_j/|r_j|)
 *   offsets  device int32 [n_env+1], offsets[0] = 0, non-decreasing,
 *            offsets[n_env] = n_nbr (neighbours of env e are
 *            offsets[e] .. offsets[e+1]-1)
 *   pos      device double [n_nbr][3] relative positions, |r_j| > 0
 *   A        device double [n_env][P1][2] (output)
 * An environment without neighbours gives A = 0.  O(3) graphs only.
 */
ace_status ace_basis(const ace_graph* g, int64_t n_env, const int32_t* offsets,
                     const double* pos, double* A, void* stream);

/*
 * Recursive contraction from given one-particle values (Sec. 2.6):
 *   phi[e]  = sum_{k in K} c_k prod_t A[e][k_t]             (Eq. (2.1))
 *   Abar[e][i] = d phi[e] / d A[e][i]  (holomorphic derivative; optional)
 *   coeffs  device double [|K|]
 *   A       device double [n_env][P1][2]
 *   phi     device double [n_env][2] (output)
 *   Abar    device double [n_env][P1][2] (output) or NULL to skip the
 *           reverse pass
 *   workspace / ws_bytes   device scratch of >= ace_workspace_size(g,
 *           n_env, 0, flags) bytes
 */
ace_status ace_contract(const ace_graph* g, const double* coeffs, int64_t n_env,
                        const double* A, double* phi, double* Abar,
                        void* workspace, size_t ws_bytes, uint32_t flags, void* stream);

/*
 * Full path: one-particle basis, recursive DAG contraction (Eq. (2.1)).
 *   phi  device double [n_env][2] = (Re phi_e, Im phi_e)
 * Other arguments as for ace_basis / ace_contract.  n_env = 0 is a no-op.
 */
ace_status ace_eval(const ace_graph* g, const double* coeffs, int64_t n_env,
                    const int32_t* offsets, const double* pos, double* phi,
                    void* workspace, size_t ws_bytes, uint32_t flags, void* stream);

/*
 * Full path with gradients: as ace_eval, plus
 *   grad device double [n_nbr][3] = d Re(phi_e) / d r_j for every neighbour
 *        j of environment e (forces are -grad)
 * computed by the reverse pass over the DAG chained into dA/dr_j.
 */
ace_status ace_eval_grad(const ace_graph* g, const double* coeffs, int64_t n_env,
                         const int32_t* offsets, const double* pos, double* phi,
                         double* grad, void* workspace, size_t ws_bytes,
                         uint32_t flags, void* stream);

/*
 * Result of the device-side validation of a call made with ACE_FLAG_CHECK
 * (ace_eval or ace_eval_grad), read from the workspace that call used, after
 * its stream has been synchronised (synchronous 4-byte copy):
 * ACE_OK if the offsets were valid; ACE_ERR_INVALID_ARG, with the reason in
 * ace_last_error(), if they were not (offsets[0] != 0 or a decrease).  The
 * check does not see offsets[n_env] against the length of pos.
 */
ace_status ace_check_offsets_result(const void* workspace);

/*
 * ace_eval_grad without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Arguments and results as for
 * ace_eval_grad; ACE_FLAG_CHECK is not accepted.  The workspace is a fixed
 * device array of 64 MiB inside the library, one per device, set up when a
 * graph is built on that device and held until the process ends; the call
 * allocates nothing.  Batches whose ace_workspace_size exceeds 64 MiB fail
 * with ACE_ERR_INVALID_ARG (split them: 4096 environments of the
 * 343-function basis n, l <= 6 fit, 8192 do not).  Every call on a device
 * shares that device's array, so calls that overlap in time on one device
 * (on any streams, from any threads) race and give wrong results: serialise
 * them.  No result depends on what an earlier call left in the array.
 */
ace_status ace_eval_grad_noalloc(const ace_graph* g, const double* coeffs, int64_t n_env,
                                 const int32_t* offsets, const double* pos, double* phi,
                                 double* grad, uint32_t flags, void* stream);

/*
 * Introspection for tests (host only, no device work).
 *
 * ace_debug_schedule: the schedule ace_eval_grad uses without flags:
 *   *kind = 1 forest (one-particle and order-2 node values resident in
 *   LDS, every higher node computed in registers), 2 remat (one-particle
 *   values resident, the two parents of every term recomputed from their
 *   one-particle factors), 0 layer by layer.  For a graph built with
 *   ACE_BUILD_HOST_ONLY the choice assumes 160 KiB of LDS per block.  When
 *   the forest is not used, ace_last_error() names the reason.  If info is
 *   not NULL it receives 16 int64 schedule sizes.  Forest: resident slots,
 *   tree slices, child positions (padded, real), pair-row slices, pair
 *   entries (padded, real), grandchildren, the four hot slots, whether all
 *   resident adjoints fit in LDS, the mean LDS bank cost of pair entries
 *   and of children (x1000), the real children plus real pair entries of
 *   the folded forest schedule (0 if it has none).  Remat: LDS value slots, then of the schedule
 *   with the adjoint slices, entry positions (padded, real), items, then of
 *   the forward-only schedule slices, entry positions (padded, real), the
 *   four hot slots, the pair slots of the schedule with the adjoint, the
 *   mean LDS bank cost of its entry reads (x1000), the entries (real)
 *   of the folded schedule with the adjoint, and the mean bank load of its
 *   row pushes (x1000: most lanes of a quarter-wave on one 8-byte bank
 *   pair, slot mod 16, per push instruction).  The rest are 0.
 *
 * ace_debug_remat_eval: as ace_debug_forest_eval for the remat schedules
 *   (phi and Abar from the one with the adjoint; ACE_ERR_INTERNAL also if
 *   the forward-only one gives another phi; ACE_ERR_UNSUPPORTED if the
 *   graph has none).  folded != 0 runs the schedules with conjugate pairs
 *   folded, which are exact only for A with A_{n,l,-m} = (-1)^m
 *   conj(A_{n,l,m}); their Abar then gives d Re(phi) as Re sum_i Abar_i dA_i
 *   for such A but is not dphi/dA itself.
 *
 * ace_debug_forest_eval: runs the forest schedule on the host for n_env
 *   environments, with the same indices, padding and forwarding as the
 *   kernel and every index bounds-checked.  coeffs [|K|], A [n_env][P1][2],
 *   phi [n_env][2], Abar [n_env][P1][2], all HOST pointers.
 *   ACE_ERR_UNSUPPORTED if the graph has no forest schedule,
 *   ACE_ERR_INTERNAL if an index of the schedule is out of range.
 *   folded != 0 runs the forest schedule with conjugate pairs folded, with
 *   the same restriction on A and the same meaning of Abar as for
 *   ace_debug_remat_eval.
 */
ace_status ace_debug_schedule(const ace_graph* g, int32_t* kind, int64_t* info);
ace_status ace_debug_forest_eval(const ace_graph* g, const double* coeffs, int64_t n_env, const double* A,
                                 double* phi, double* Abar, int32_t folded);
ace_status ace_debug_remat_eval(const ace_graph* g, const double* coeffs, int64_t n_env, const double* A,
                                double* phi, double* Abar, int32_t folded);

#ifdef __cplusplus
}
#endif

#endif /* ACE_H_ */
