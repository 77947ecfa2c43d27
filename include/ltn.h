/*
 * ltn.h -- C ABI of the sliced tensor-network contraction library (libltn).
 *
 * The library evaluates amplitudes of a random quantum circuit by
 * contracting its tensor network along a contraction tree with a set of
 * sliced edges, after Chen et al., "Lifetime-based Optimization for
 * Simulating Quantum Circuits on a New Sunway Supercomputer" (PPoPP'23):
 *
 *   network G = (V, E), w(e) = 2              (Sec. 2.1.1, Notation)
 *   contraction path / rooted binary tree B   (Sec. 2.1.1)
 *   slicing set S, 2^|S| independent subtasks whose results are summed
 *                                             (Sec. 2.1.1, Eq. (2))
 *   slice finder on the stem                  (Sec. 4.2, Algorithm 1)
 *
 * Conventions shared by every call:
 *   - complex numbers are interleaved (re, im); complex64 = 2 x float,
 *     complex128 = 2 x double;
 *   - a tensor of rank r is a dense array of 2^r elements, row-major over
 *     its index list (the first index is the slowest);
 *   - an "index id" is an edge of the network, 0 <= id < n_indices;
 *   - SSA path: leaves are 0..L-1, the k-th contraction creates id L+k;
 *     path[2k], path[2k+1] are its two operands;
 *   - slice id s: bit j (LSB = 0) of s is the value of the sliced index
 *     S[j]; slice ids are 64-bit, so when |S| > 64 the indices S[64..]
 *     keep the value 0 (the addressable slices are the first 2^64);
 *   - output vector: one entry per assignment of the open indices, the
 *     first open index is the most significant bit; sliced open indices
 *     take their bits from the slice id (placement), the others are summed
 *     over slices.
 *
 * Errors: every call returns an ltn_status; 0 is success, negative values
 * are errors and ltn_last_error() returns a message (thread-local, valid
 * until the next failing call on the same thread). No exception crosses
 * the ABI. Host arrays passed in are borrowed for the duration of the call
 * and copied. Device buffers passed in are owned by the caller and must
 * outlive the stream work that uses them.
 */
#ifndef LTN_H
#define LTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ltn_status;
enum {
  LTN_OK = 0,
  LTN_E_INVALID = -1, /* malformed input (shape, id, path, slice id ...)   */
  LTN_E_CAP = -2,     /* a tensor's rank after slicing exceeds max_rank    */
  LTN_E_NOMEM = -3,   /* workspace too small for one slice                 */
  LTN_E_HIP = -4,     /* a HIP runtime call failed (message has the code)  */
  LTN_E_STATE = -5,   /* call not valid in the plan's state (e.g. unbound) */
  LTN_E_UNSUPPORTED = -6
};

/* Precision of the contraction steps (all accumulate in FP32 and sum the
 * slices in FP64). In the split modes every step that takes the MFMA GEMM
 * with at least 8 contracted complex elements splits each real part of
 * both operands, scaled by an exact power of two, into hi + lo in fp16
 * (11 + 11 bits) or bf16 (8 + 8 bits) and sums hi*hi, hi*lo and lo*hi on
 * the matrix cores; the other steps stay complex64. Tensors stay complex64
 * in memory. */
enum {
  LTN_C64 = 0,        /* complex64 GEMMs on FP32 MFMA / FP32 VALU          */
  LTN_SPLIT_F16 = 1,  /* each real part split into fp16 hi + lo (scaled)   */
  LTN_SPLIT_BF16 = 2  /* each real part split into bf16 hi + lo (scaled)   */
};

/* ------------------------------------------------------------------------
 * Circuits and networks (host).
 * ---------------------------------------------------------------------- */

/* Gate kinds of the synthetic random circuits. Matrices are [out][in];
 * two-qubit gates act on |q0 q1> with q0 the more significant qubit. */
enum {
  LTN_GATE_SQRT_X = 1, /* ((1+i)/2) I + ((1-i)/2) X                       */
  LTN_GATE_SQRT_Y = 2, /* ((1+i)/2) I + ((1-i)/2) Y                       */
  LTN_GATE_SQRT_W = 3, /* ((1+i)/2) I + ((1-i)/2) W, W = (X+Y)/sqrt 2     */
  LTN_GATE_FSIM = 4,   /* fsim(theta = p[0], phi = p[1])                   */
  LTN_GATE_U3 = 5,     /* Rz(p[0]) Ry(p[1]) Rz(p[2]), a parameterised leaf */
  LTN_GATE_MATRIX = 6  /* explicit 2x2 or 4x4 complex128 matrix in m[]     */
};

typedef struct ltn_gate {
  int32_t kind;
  int32_t q0, q1;   /* q1 = -1 for single-qubit gates                      */
  int32_t param_id; /* u3 gates: 0.. in circuit order; -1 otherwise        */
  double p[3];
  double m[32];     /* LTN_GATE_MATRIX: row-major complex128 (re, im)      */
} ltn_gate;

/* A tensor network, as consumed by the planner and by ltn_plan_load.
 * Every index must lie in exactly two leaves (closed) or exactly one leaf
 * (open; then it must be listed in open_ids). */
typedef struct ltn_network {
  int32_t n_leaves;
  const int64_t* leaf_off;  /* [n_leaves+1] CSR offsets into index_ids    */
  const int32_t* index_ids; /* per leaf, axis order (first = slowest)     */
  const float* leaf_data;   /* complex64 data of each leaf, concatenated
                               in leaf order, 2^rank elements each; the
                               data of parameterised leaves is ignored    */
  int32_t n_open;
  const int32_t* open_ids;  /* output order, first = most significant     */
  int32_t n_indices;
  const int32_t* param_leaf; /* [n_leaves] u3 gate id or -1; may be NULL  */
} ltn_network;

typedef struct ltn_netbuf ltn_netbuf; /* an owned network built by the library */

/* Build the network <b| C |0> of a circuit (gates in order) and absorb its
 * non-parameterised rank-1 and rank-2 tensors (Sec. 2.1.2: preprocessing
 * "rank-1 and rank-2 tensors are absorbed"). closed_bits[q] is the fixed
 * output bit of qubit q, or -1 for an open qubit (open indices are listed
 * in ascending qubit order). Index ids are given in creation order (the
 * initial wire of qubit q is id q, then every gate creates one id per
 * qubit it acts on); tensors are |0> per qubit, the gates, then <b_q| per
 * closed qubit. Absorption repeatedly merges the lowest-id tensor of rank
 * <= 2 that is not a u3 leaf into its lowest-id non-u3 neighbour (axes:
 * the neighbour's unshared axes, then the absorbed tensor's), in
 * complex128, then rounds to complex64; ids are then renumbered densely.
 * absorb = 0 skips absorption. */
ltn_status ltn_network_build(int32_t n_qubits, const ltn_gate* gates, int32_t n_gates,
                             const int32_t* closed_bits, int32_t absorb, ltn_netbuf** out);
/* Fill *view with pointers into the netbuf (valid until ltn_netbuf_free). */
ltn_status ltn_netbuf_view(const ltn_netbuf* nb, ltn_network* view);
/* complex128 leaf data (before rounding), concatenated like leaf_data. */
ltn_status ltn_netbuf_data128(const ltn_netbuf* nb, const double** data);
void ltn_netbuf_free(ltn_netbuf* nb);

/* ------------------------------------------------------------------------
 * Host planner: path, tree costs, lifetimes, slice finder.
 * ---------------------------------------------------------------------- */

/* Greedy contraction path. Among pairs of live tensors that share an index
 * (ignoring the indices in `exclude`), contract the pair with the smallest
 * key; when no pair shares an index, join the two lowest ids.
 *   key = (2^rc - alpha (2^ra + 2^rb)) * (1 + tau u)  if the bracket > 0
 *         (2^rc - alpha (2^ra + 2^rb)) * (1 - tau u)  otherwise
 * evaluated in IEEE double in that order (rc, ra, rb = ranks of the result
 * and operands), with u in [0,1) from SplitMix64 keyed by (seed, step, a,
 * b); ties go to the smallest (lower id, higher id). tau = 0, alpha = 1 is
 * the plain greedy rule. path_out: [2*(L-1)]. */
ltn_status ltn_greedy_path(const ltn_network* net, const int32_t* exclude, int32_t n_exclude,
                           double alpha, double tau, uint64_t seed, int32_t* path_out);

/* Costs of a tree with slicing set S (exact integers as little-endian
 * 64-bit words, and their log2):
 *   cost      = Eq. (1) C(B), summed over the contraction nodes;
 *   sliced    = Eq. (4) C(B,S);
 *   space     = log2 of the largest tensor after slicing;
 *   overhead  = Eq. (2) C(B,S) / C(B). */
typedef struct ltn_costs {
  double log2_cost, log2_sliced, overhead;
  int32_t space_log2, space_log2_unsliced;
  uint64_t cost_words[4];
  uint64_t sliced_words[4];
  int32_t stem_len;
} ltn_costs;
ltn_status ltn_tree_costs(const ltn_network* net, const int32_t* path, const int32_t* S,
                          int32_t n_sliced, ltn_costs* out);

/* Stem of the tree (Sec. 4.2): the root-to-leaf path of largest summed
 * Eq. (1) node cost, as node ids ordered leaf -> root (ties: larger
 * subtree cost, then smaller id). stem_out capacity = cap. */
ltn_status ltn_tree_stem(const ltn_network* net, const int32_t* path, int32_t* stem_out,
                         int32_t cap, int32_t* len);

/* Profile of the stem (Sec. 4.2), one row per stem tensor from the leaf to
 * the root: its node id, its rank, its rank after removing the indices in
 * S, and log2 of the Eq. (1) cost of the contraction that produces it
 * (|s_v1 u s_v2 u s_v3|, the node's index set) without and with S (-1 for
 * the leaf). rows capacity = cap; *len = number of stem tensors. Host only.
 * Errors: LTN_E_NOMEM if cap is below the stem length. */
typedef struct ltn_stem_row {
  int32_t tensor, rank, rank_sliced, node_bits, node_bits_sliced;
} ltn_stem_row;
ltn_status ltn_stem_profile(const ltn_network* net, const int32_t* path, const int32_t* S,
                            int32_t n_sliced, ltn_stem_row* rows, int32_t cap, int32_t* len);

/* Lifetime-based slice finder (Sec. 4.2, Algorithm 1) under target rank t,
 * starting from the indices in `pre` (already sliced; the tree, its stem
 * and the lifetimes are taken without them). Ranks are counted after the
 * current S. The stem tensors above t are fixed from the ends of their
 * stretch inwards: each round takes the end tensor of smaller rank (the
 * root-side one on a tie) and slices as many of its unsliced indices as it
 * exceeds t by, preferring the index whose stem lifetime (an interval of
 * stem positions) covers the most over-cap stem tensors, then the one held
 * by the most tree tensors, then the smaller id; tensors that now fit
 * leave the stretch. A fix-up then slices, for every tree tensor still
 * above t (SSA order), its unsliced index held by the most tree tensors
 * (then the smaller id). t < 0 means no cap (S = pre). S_out receives pre
 * followed by the added indices (capacity cap). */
ltn_status ltn_slice_finder(const ltn_network* net, const int32_t* path, int32_t t,
                            const int32_t* pre, int32_t n_pre, int32_t* S_out, int32_t cap,
                            int32_t* n_sliced);

/* Randomised greedy search: for every (alpha, tau, seed) trial below, run
 * ltn_greedy_path then ltn_slice_finder, and keep the trial with the
 * smallest (C(B,S), |S|, trial number). Trials are numbered alpha-major,
 * then tau, then seed (0..n_seeds-1); trials with tau = 0 use seed 0 only.
 * With reconf_k >= 3 every trial's path is improved before and after the
 * slice finder by ltn_tree_reconfigure (k = reconf_k, reconf_sweeps sweeps;
 * first with S = pre and no cap, then with the trial's S under the cap t).
 * reconf_k = 0 leaves the greedy paths as they are. */
typedef struct ltn_search_opts {
  int32_t n_alpha;
  const double* alphas;
  int32_t n_tau;
  const double* taus;
  int32_t n_seeds;
  uint64_t seed_base;
  int32_t reconf_k;
  int32_t reconf_sweeps;
} ltn_search_opts;
ltn_status ltn_path_search(const ltn_network* net, int32_t t, const int32_t* pre, int32_t n_pre,
                           const ltn_search_opts* opts, int32_t* path_out, int32_t* S_out,
                           int32_t cap, int32_t* n_sliced, int32_t* best_trial);

/* Slice refiner (Sec. 4.3, Algorithms 2-4): simulated annealing over edge
 * replacements at fixed |S|. Each iteration picks a slot of S (beyond the
 * first n_fixed, which never move) with a keyed uniform draw; the critical
 * tensors of its index are the tensors holding it (leaves included) whose
 * rank after S equals t (Algorithm 3); the candidates are the unsliced
 * indices whose lifetime contains all of them (Sec. 4.3; the set Algorithm 4
 * forms by intersecting their index sets), tried in ascending id, each
 * replacing the slot's current occupant: a move that lowers C(B,S) (Eq. 4)
 * is taken, a costlier one with probability exp((C_ori - C_new)/C_ori/T).
 * An index with no critical tensor in its lifetime is dropped from S. T
 * starts at t0 and is multiplied by alpha every iters_per_temp iterations
 * until T < tf. Draws: slot = n_fixed + floor(u (|S| - n_fixed)) with
 * u = keyed_uniform(seed, iteration, 0, 0); uphill acceptance draws
 * keyed_uniform(seed, iteration, 1, candidate id) (SplitMix64 keyed as in
 * ltn_greedy_path). Every set it visits meets the cap; the best seen (lowest
 * C(B,S), first reached) is returned in S_out (capacity n_in; the order of
 * kept slots is preserved, so bit j of a slice id stays the value of S[j]).
 * Errors: LTN_E_CAP if S_in does not meet the cap t; LTN_E_INVALID for a
 * repeated id or bad parameters (alpha outside (0,1), non-positive t0/tf,
 * iters_per_temp < 1, n_fixed outside 0..n_in). */
typedef struct ltn_refine_opts {
  double t0;              /* initial temperature (1.0)                     */
  double alpha;           /* cooling factor (0.98)                         */
  double tf;              /* final temperature (1e-3)                      */
  int32_t iters_per_temp; /* iterations at each temperature (1)            */
  int32_t n_fixed;        /* leading entries of S that are never replaced  */
  uint64_t seed;
} ltn_refine_opts;
typedef struct ltn_refine_stats {
  int32_t iterations, proposals, accepted, dropped;
} ltn_refine_stats;
ltn_status ltn_slice_refine(const ltn_network* net, const int32_t* path, int32_t t,
                            const int32_t* S_in, int32_t n_in, const ltn_refine_opts* opts,
                            int32_t* S_out, int32_t* n_out, ltn_refine_stats* stats);

/* Subtree reconfiguration of a contraction tree (a path improvement in the
 * spirit of the local tuning of the tree between slicing steps named in
 * Sec. 2.1.2). Each sweep visits every contraction node v in SSA order: a
 * frontier grows from v by replacing the frontier node with the largest
 * node set (Eq. 1's s_v without the indices in S; ties: smaller id) by its
 * two children, up to k tensors (k in 2..16); the frontier is re-contracted
 * in the order of least summed node cost 2^|s_v - S| found by exhaustive
 * search over its subsets (with t >= 0, no intermediate tensor may exceed
 * rank t after S; t < 0: no cap), and the new subtree is kept when strictly
 * cheaper. Costs saturate at 2^120. After each sweep the tree is written
 * out again as an SSA path in post order (left child first); sweeps stop
 * early when one changes nothing. path_out: 2 (n_leaves - 1) ids, may not
 * alias path. With S empty this lowers Eq. (1); with S and t it lowers
 * Eq. (4) while every tensor stays within the cap. */
ltn_status ltn_tree_reconfigure(const ltn_network* net, const int32_t* path, int32_t k,
                                int32_t sweeps, const int32_t* S, int32_t n_sliced, int32_t t,
                                int32_t* path_out);

/* Greedy least-overhead slicer, the strategy the paper attributes to
 * cotengra (Sec. 2.1.2), for comparison with Algorithm 1: starting from pre,
 * while some tree tensor has rank > t after S, append the unsliced index of
 * such tensors that gives the smallest C(B,S) (Eq. 4); ties: held by the
 * most tensors above t, then the smaller id. S_out capacity = cap. */
ltn_status ltn_slice_greedy_overhead(const ltn_network* net, const int32_t* path, int32_t t,
                                     const int32_t* pre, int32_t n_pre, int32_t* S_out,
                                     int32_t cap, int32_t* n_sliced);

/* ------------------------------------------------------------------------
 * Plans and execution.
 * ---------------------------------------------------------------------- */

typedef struct ltn_plan ltn_plan;

typedef struct ltn_options {
  int32_t max_rank;      /* cap check t: every tensor after slicing must
                            have rank <= max_rank (negative: no check)     */
  int32_t batch;         /* slices per batch; 0 = as many as fit          */
  int32_t fat_threshold; /* steps with min(k, n, m) bits >= this go to the
                            MFMA GEMM (0 = library default)                */
  int32_t fuse_rank;     /* > 0: fuse runs of stem steps that absorb small
                            tensors (secondary slicing, Sec. 5.2) when every
                            working tensor has rank <= fuse_rank (<= 11);
                            0 = no fusion                                   */
} ltn_options;

/* Compile a plan (host only, no device call) for the problem as Sec. 2.1.1
 * states it: a network G (every edge of weight 2), a contraction tree B
 * given by an SSA path, and a slicing set S whose 2^|S| value assignments
 * are independent subtasks. Validate the network, the
 * SSA path and the slicing set, assign every tensor its layout (unsliced
 * indices sorted by the step that contracts them, earliest = lowest bit;
 * open indices last, in output order; since an index shared by the two
 * operands of a contraction is absent from its result (Lemma 1,
 * supplement), the summed indices are the lowest bits of both operands and
 * every step is a GEMM without operand transposition), give every step its
 * (m, k, n) bit groups and kernel (per slice the steps' multiply-adds sum to
 * C(B,S) / 2^|S|, Eq. (4)), and lay tensors out in a per-slice arena by
 * liveness; no tensor exceeds 2^t elements when max_rank = t (the memory
 * bound of Sec. 4.1).
 * Errors: LTN_E_INVALID (index in more than two leaves, open index not
 * listed, path not an SSA cover, duplicate / unknown sliced id, more than
 * 255 sliced indices, a tensor of rank > 40 after slicing), LTN_E_CAP
 * (max_rank exceeded). */
ltn_status ltn_plan_load(const ltn_network* net, const int32_t* path_ssa, int32_t n_sliced,
                         const int32_t* sliced_ids, const ltn_options* opt, ltn_plan** out);

typedef struct ltn_plan_info {
  int32_t n_leaves, n_steps, n_sliced, n_open, n_open_unsliced, n_params;
  int32_t batch;                /* 0 until bound                          */
  int32_t root_rank;
  double macs_per_slice;        /* sum over steps of 2^(m+k+n)            */
  uint64_t macs_words[2];       /* the same, exact                        */
  uint64_t arena_bytes_per_slice;
  uint64_t grad_arena_bytes_per_slice;
  uint64_t const_bytes;         /* batch-independent part of a workspace  */
  const int32_t* sliced_ids;    /* [n_sliced], bit order of slice ids     */
} ltn_plan_info;
ltn_status ltn_plan_describe(const ltn_plan* plan, ltn_plan_info* out);

/* Fused sub-paths of a plan (secondary slicing, Sec. 5.2): group g covers
 * the chain steps first_step[g] .. (in chain order, n_steps[g] of them; the
 * last one is where it runs), fixes the |Sigma| = n_sigma[g] indices of its
 * input that survive to its output, and works on tensors of at most
 * 2^work_rank[g] elements per piece. Arrays of capacity cap; *n = number
 * of groups. Host only. */
ltn_status ltn_plan_groups(const ltn_plan* plan, int32_t* first_step, int32_t* n_steps,
                           int32_t* n_sigma, int32_t* work_rank, int32_t cap, int32_t* n);

/* Run fused sub-paths (enable != 0, the default after ltn_bind) or step
 * by step in the forward pass of ltn_execute / ltn_execute_range. Gradient
 * passes always run step by step (the adjoint reads every intermediate).
 * Drops captured graphs. Errors: LTN_E_STATE if unbound. */
ltn_status ltn_set_fusion(ltn_plan* plan, int32_t enable);

/* Kernel classes a step can use. */
enum { LTN_K_SMALL = 0, LTN_K_MFMA = 1 };

typedef struct ltn_step_info {
  int32_t left, right, out; /* SSA ids                                      */
  int32_t a_is_left;        /* operand A (rows m) is the left SSA operand   */
  int32_t m, k, n;          /* bits of the free-A, contracted, free-B groups */
  int32_t kernel;           /* LTN_K_*                                       */
  const int32_t* a_idx;     /* A's unsliced indices, lowest bit first       */
  const int32_t* b_idx;     /* B's unsliced indices, lowest bit first       */
  const int32_t* c_idx;     /* the output's indices, lowest bit first       */
  uint64_t c_mask_a;        /* output bits that come from A (rest from B)   */
  uint64_t arena_off_a, arena_off_b, arena_off_c; /* per-slice byte offsets */
} ltn_step_info;
ltn_status ltn_plan_step(const ltn_plan* plan, int32_t step, ltn_step_info* out);

/* Bytes of workspace for `batch` slices per batch (grad != 0: enough for
 * ltn_execute_grad as well): leaf data and descriptors, then per slice the
 * arena of the tensors live at once (each at most 2^t complex64 elements
 * under the cap t of Sec. 4.1), split-precision operand copies and
 * split-sum partials. The paper keeps each subtask's tensors in one
 * process's memory (Sec. 4.1, Sec. 5.2); how a device holds several
 * slices at once is this library's. Host only. Errors: LTN_E_INVALID for
 * batch < 1. */
ltn_status ltn_workspace_size(const ltn_plan* plan, int32_t batch, int32_t grad, size_t* bytes);

/* Bind device memory and a HIP stream (hipStream_t passed as void*; NULL =
 * the default stream). The paper has no counterpart (its subtasks run in
 * separate processes, Sec. 6.1); here several slices of one plan are
 * resident at once and run in the same launches. d_workspace is caller-
 * owned device memory of `bytes` bytes, 256-byte aligned, that must stay
 * allocated until the plan is freed or bound again; the plan keeps its own
 * captured graphs. The batch size becomes the largest that fits in
 * `bytes` (capped by ltn_options.batch when set); the grad flag must match
 * the one used for ltn_workspace_size. Uploads leaf data (async on the
 * stream). Errors: LTN_E_NOMEM if not even one slice fits. */
ltn_status ltn_bind(ltn_plan* plan, void* d_workspace, size_t bytes, int32_t grad, void* stream);

/* Contract the listed slices (host array of n ids, each < 2^|S| when
 * |S| < 64) and ADD the result into d_out (complex128, 2^n_open entries,
 * caller-owned device memory). Each slice is one of the 2^|S| independent
 * subtasks of Sec. 2.1.1 and the subtasks' results are accumulated, as
 * there; the paper's processes meet in one allReduce at the end (Sec.
 * 6.1), so d_out is only ever added to (the caller zeroes it), which lets
 * partitioned id lists and ranges be summed.
 * Slices are summed in FP64, in batches of the bound batch size; within a
 * batch in ascending position, batches in call order. Asynchronous on the
 * bound stream, except that the first call in a mode after ltn_bind, a
 * kernel choice or a fusion change synchronises it once (the launch
 * descriptors of that mode are uploaded and a graph is captured). On a
 * plan bound with grad != 0, a complex64 call of at most one batch runs in
 * the gradient arena and its intermediates stay there for a following
 * ltn_execute_grad on the same ids (see there). Errors:
 * LTN_E_STATE (unbound), LTN_E_INVALID (bad id / mode). */
ltn_status ltn_execute(ltn_plan* plan, const uint64_t* slice_ids, uint64_t n, int32_t mode,
                       void* d_out);
/* Same for the slice ids begin .. end-1 (end <= 2^|S| when |S| < 64;
 * LTN_E_INVALID otherwise or when end < begin). */
ltn_status ltn_execute_range(ltn_plan* plan, uint64_t begin, uint64_t end, int32_t mode,
                             void* d_out);

/* Size of the library's own device scratch array (one per GPU, held until
 * the process ends), used by ltn_execute_scratch. */
#define LTN_SCRATCH_BYTES (64u << 20)

/* ltn_execute for callers that cannot allocate device memory or bind a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): contracts the listed slices of a loaded plan
 * (bound or not; its own binding is left as it is) in the library's
 * scratch array of LTN_SCRATCH_BYTES on the current device, and ADDS the
 * result into d_out (complex128, 2^n_open entries, device), with the same
 * arithmetic and summation order as ltn_execute for the batch size that
 * fits (as many slices per batch as the scratch holds, at most n). Leaf
 * data and descriptors are uploaded at every call; batches run eagerly
 * (no graphs), with the default kernel choices, on `stream` (hipStream_t
 * as void*; NULL = default stream); the call returns once its uploads are
 * done and its kernels are enqueued. It allocates nothing: no hipMalloc,
 * hipFree or allocating library routine. Every call on one GPU uses that
 * GPU's one scratch array, so calls that overlap on one GPU (other host
 * threads, other streams) race and must be serialised by the caller; the
 * array keeps the last call's contents, and whatever must start at zero is
 * cleared by the call itself. Errors: LTN_E_NOMEM if one slice needs more
 * than LTN_SCRATCH_BYTES, LTN_E_INVALID (NULL argument, bad id or mode). */
ltn_status ltn_execute_scratch(ltn_plan* plan, const uint64_t* slice_ids, uint64_t n, int32_t mode,
                               void* d_out, void* stream);

/* The paper has no parameterised gates or gradients; this call and
 * ltn_execute_grad extend the same sliced contraction to rotation angles.
 * Rebuild every parameterised (u3) leaf from angles on the device:
 * d_angles is float64 [n_params] laid out [gate][a, b, c] with
 * U = Rz(a) Ry(b) Rz(c). Asynchronous on the bound stream. */
ltn_status ltn_set_params(ltn_plan* plan, const double* d_angles);

/* Gradient of a real loss with respect to the u3 angles, by an adjoint
 * contraction (not in the paper): each slice stays an independent subtask
 * (Sec. 2.1.1), its forward contraction is recomputed, each step's two
 * cotangents are the conjugate products of the output cotangent with the
 * other operand, and leaf cotangents are summed over slices in FP64 before
 * the u3 chain rule. d_cotangent is the loss gradient with respect to the
 * output vector (complex128, 2^n_open entries, PyTorch convention
 * dL/dRe + i dL/dIm). Adds the forward result into d_out (may be NULL) and
 * dL/dangle into d_angle_grad (float64 [n_params]); all three are
 * caller-owned device memory. Asynchronous on the bound stream, except that
 * the first call after ltn_bind or a kernel choice change synchronises it
 * once (launch descriptors uploaded, graphs captured). When the previous
 * call on the plan was a one-batch complex64 ltn_execute of the same id
 * list (and ltn_set_params was not called since), its intermediates are
 * still in the gradient arena and the forward is not recomputed; any other
 * call in between drops them. Errors: LTN_E_STATE
 * if the plan is not bound with grad != 0, LTN_E_INVALID for a bad id or
 * mode, LTN_E_UNSUPPORTED for the split modes (complex64 only). */
ltn_status ltn_execute_grad(ltn_plan* plan, const uint64_t* slice_ids, uint64_t n, int32_t mode,
                            const void* d_cotangent, void* d_out, double* d_angle_grad);

/* Time every distinct step shape with the candidate kernel configurations
 * on the bound stream and keep the fastest (cached in `cache_path` as JSON
 * when non-NULL). In complex64 mode on a plan bound with grad != 0, the
 * adjoint products of the gradient sweep (the forward-form GEMMs of
 * ltn_execute_grad) are tuned as well: every complex64 tile and, for sums
 * of 2^10 and more, every split-K tile that fits each product shape in
 * either operand role, against the fixed rule (cache keys g0_m_k_n_bB,
 * values [1000 kind + cfg, swap] or [-1, 0]; a cached choice that does not
 * fit its shape falls back to the fixed rule). (Kernel choice is not part
 * of the paper's method.) Synchronises the stream. */
ltn_status ltn_autotune(ltn_plan* plan, int32_t mode, const char* cache_path);

/* Per-step timing of one batch (debug replay outside the graph): writes
 * n_steps floats of milliseconds into ms_out. Synchronises the stream. */
ltn_status ltn_profile_steps(ltn_plan* plan, uint64_t first_slice, int32_t mode, float* ms_out);

/* Bit permutation of a batch of complex64 tensors (the layout change a
 * transpose-transpose-GEMM-transpose contraction applies around each GEMM,
 * Sec. 2.1.2 and Sec. 5.3.1; the plan's own steps never need it because
 * their layouts make every operand GEMM-ready and fold the output
 * transposition into the GEMM's store):
 *     out[b][y] = in[b][x]   with bit perm[j] of y equal to bit j of x
 * (bit 0 = fastest-varying). d_in / d_out: device complex64 arrays of
 * batch * 2^rank elements, tensor b at offset b * 2^rank, 16-byte aligned
 * when rank >= 1; they must not overlap. perm: host array of rank entries,
 * a permutation of 0..rank-1. Staged through LDS tiles that cover the
 * lowest 5 bits of both sides, so reads and writes are coalesced (16 bytes
 * per lane). Asynchronous on `stream` (hipStream_t as void*; NULL = default
 * stream). Errors: LTN_E_INVALID (rank > 40, perm not a permutation,
 * in == out, batch < 1, a buffer not 16-byte aligned). */
ltn_status ltn_permute(const void* d_in, void* d_out, int32_t rank, const int32_t* perm,
                       int64_t batch, void* stream);

/* Kernel chosen for a step in a mode after ltn_bind / ltn_autotune:
 * kind 0 = generic VALU kernel (tk threads per output), 1 = complex64 MFMA
 * GEMM, 2 = split-precision MFMA GEMM, 3 = narrow-step kernel (cfg 0:
 * k + n <= 10, n <= 6, A tile in LDS, B broadcast from LDS, outputs staged
 * in address order; cfg 1: k, n <= 4, m >= 8, one thread per row of A with
 * all its loads in flight, B broadcast from LDS), 4 = split-sum kernel for steps with few outputs (m <= 3, n <= 3:
 * the sum over k is cut into chunks reduced by separate blocks, FP32
 * partials added in FP32 in a fixed order), 5 = split-K complex64 MFMA GEMM
 * (sums of 2^10 and more cut into chunks that separate blocks reduce on the
 * matrix cores, tiles down to 16 complex columns, FP32 partials added in
 * chunk order by a second pass); cfg = tile configuration of that
 * kind (-1 for the generic kernel); swap = operands exchanged (rows come
 * from B). Requires a bound plan. */
/* Force the kernel of one step in one mode (same encoding as
 * ltn_step_kernel; tk in {1, 8, 64} for kind 0). Errors: LTN_E_INVALID if
 * the kernel does not fit the step (tile too large, narrow or split-sum
 * limits) or a
 * split kind is asked for in complex64 mode; LTN_E_STATE if unbound. The
 * plan's captured graphs are dropped. */
ltn_status ltn_set_step_kernel(ltn_plan* plan, int32_t step, int32_t mode, int32_t kind,
                               int32_t cfg, int32_t swap, int32_t tk);

ltn_status ltn_step_kernel(const ltn_plan* plan, int32_t step, int32_t mode, int32_t* kind,
                           int32_t* cfg, int32_t* swap, int32_t* tk);

/* Name of a kernel choice (kind and cfg as in ltn_step_kernel) in a mode,
 * e.g. "c64_3m_128x64x32": a static string, "?" for a choice that does not
 * exist. Complex64 tiles named c64_3m_* (kind 1) and splitk_3m_* (kind 5)
 * form each complex product from three real products (Gauss's method:
 * Re = ArBr - AiBi, Im = (Ar + Ai)(Br + Bi) - ArBr - AiBi), the others from
 * the four of the 2x2 real form; the paper does not fix how a complex
 * product is formed. Host only: needs no plan and no GPU. */
const char* ltn_kernel_name(int32_t kind, int32_t cfg, int32_t mode);

void ltn_plan_free(ltn_plan* plan);
const char* ltn_last_error(void);
const char* ltn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LTN_H */
