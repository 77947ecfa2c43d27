// Compiled plan: what ltn_plan_load derives from (network, path, S).
//
// Layout rule: every tensor stores its unsliced indices ordered by the step
// that contracts them, earliest lowest (bit 0 = fastest); ties by index id;
// open indices come last, the last open index lowest, so the root tensor is
// already in output order. With this rule the indices contracted at a step
// are the lowest bits of both operands, so every step is
//     C[merge(m, n)] = sum_k A[m * 2^k + k] * B[n * 2^k + k]
// with no input transposition; the output order is a merge of A's and B's
// free bits (each keeping its order), described by one bit mask.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "common.h"

struct LeafPlan {
  int32_t leaf = 0;
  int32_t tensor = 0;          // tensor id (== SSA id)
  int64_t src_off = 0;         // element offset in the leaf-data area
  int32_t rank_src = 0;        // rank as given
  int32_t rank = 0;            // unsliced rank
  std::vector<int32_t> src_bit;     // canonical bit j -> source bit position
  std::vector<int32_t> sl_src_bit;  // sliced axes: source bit position
  std::vector<int32_t> sl_bit;      //              and slice-id bit
  int32_t param = -1;
};

struct TensorPlan {
  int32_t rank = 0;
  ltn::IdSet idx;              // canonical order, lowest bit first
  uint64_t off = 0;            // forward arena, per-slice byte offset
  uint64_t goff = 0;           // grad arena: tensor
  uint64_t gcot = 0;           // grad arena: its cotangent
  int32_t producer = -1;       // step, -1 for leaves
  int32_t consumer = -1;       // step, -1 for the root
  uint64_t bytes() const { return 8ull << rank; }
};

struct StepPlan {
  int32_t left = 0, right = 0, out = 0;
  int32_t a = 0, b = 0;        // SSA ids of the row operand A and of B
  int32_t a_is_left = 1;
  int32_t m = 0, k = 0, n = 0;
  int32_t kernel = 0;
  uint64_t c_mask_a = 0;
};

// A fused sub-path (secondary slicing): consecutive stem steps s_1..s_L in
// which the chain tensor T_{j-1} meets a small tensor Y_j and becomes T_j.
// The indices of T_0 that survive to T_L are never touched inside, so fixing
// them (Sigma: all of them except the earliest-contracted ones, which are
// carried along to fill the working rank and to make writes contiguous)
// splits the sub-path into 2^|Sigma| independent pieces; each works on
// W_j = T_j without Sigma (at most 2^fuse_rank elements).
constexpr int kMaxFuseStages = 16;
struct FuseStage {
  int32_t step = 0;
  int32_t other = 0;        // SSA id of Y_j
  int32_t m = 0, k = 0, n = 0;  // W_{j-1} = [2^m][2^k] rows, Y_j = [2^n][2^k]
  uint64_t cmask = 0;       // positions in W_j of the bits from W_{j-1}
};
struct FuseGroup {
  int32_t t0 = 0, tl = 0;   // SSA ids of T_0 and T_L
  int32_t a = 0;            // low bits of T_0 that are not in Sigma
  int32_t nsig = 0;         // |Sigma|
  int32_t c = 0;            // rank of W_L
  int32_t rmax = 0;         // largest W_j rank
  int32_t b_elems = 0;      // sum of 2^rank(Y_j)
  uint64_t sig_out = 0;     // positions of the Sigma bits in T_L
  uint64_t w_out = 0;       // positions of the W_L bits in T_L
  std::vector<FuseStage> st;
};

struct ltn_plan_impl;

struct ltn_plan {
  // host description
  int32_t L = 0;
  int32_t n_indices = 0;
  std::vector<int32_t> sliced;       // S, bit order
  std::vector<int32_t> open_ids;
  std::vector<LeafPlan> leaves;
  std::vector<TensorPlan> tensors;   // by SSA id
  std::vector<StepPlan> steps;
  std::vector<int32_t> leaf_param;   // leaf -> u3 gate id
  std::vector<float> leaf_data;      // complex64, leaves concatenated
  int64_t leaf_elems = 0;
  int32_t n_params = 0;              // number of angles (3 per u3 gate)
  int32_t root = 0;
  uint64_t out_mask = 0;             // output bits filled by the root
  std::vector<std::pair<int32_t, int32_t>> out_sliced;  // (slice bit, output bit)
  int32_t n_open = 0;
  uint64_t arena = 0, garena = 0;    // per-slice bytes
  uint64_t split_scratch = 0;        // per-slice bytes for split-layout operand copies
  ltn::BigSum macs;
  double macs_d = 0;
  ltn_options opt{};
  std::vector<FuseGroup> groups;     // fused sub-paths (ltn_options.fuse_rank > 0)
  std::vector<int32_t> step_group;   // per step: its group, or -1
  // device side (runtime)
  ltn_plan_impl* rt = nullptr;
};

void runtime_free(ltn_plan* p);
void runtime_describe(const ltn_plan* p, ltn_plan_info* o);
