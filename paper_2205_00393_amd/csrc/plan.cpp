// ltn_plan_load: validation, layouts, steps, liveness-based arena.
#include "plan.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <map>
#include <memory>

using namespace ltn;

namespace {

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// First-fit offsets for blocks alive on closed time intervals.
struct Block {
  uint64_t off, size;
  int32_t end;
};
uint64_t place_block(std::vector<Block>& live, uint64_t size, int32_t begin, int32_t end,
                     uint64_t& high) {
  live.erase(std::remove_if(live.begin(), live.end(), [&](const Block& b) { return b.end < begin; }),
             live.end());
  std::sort(live.begin(), live.end(), [](const Block& a, const Block& b) { return a.off < b.off; });
  uint64_t a = std::min<uint64_t>(size, kAlign);
  uint64_t cur = 0;
  for (const Block& b : live) {
    if (align_up(cur, a) + size <= b.off) break;
    cur = std::max(cur, b.off + b.size);
  }
  uint64_t off = align_up(cur, a);
  live.push_back({off, size, end});
  high = std::max(high, off + size);
  return off;
}

}  // namespace

extern "C" ltn_status ltn_plan_load(const ltn_network* net, const int32_t* path_ssa,
                                    int32_t n_sliced, const int32_t* sliced_ids,
                                    const ltn_options* opt, ltn_plan** out) {
  return guarded([&] {
    require(out != nullptr, "out is NULL");
    Net n = Net::from_abi(net, true);
    require(net->leaf_data != nullptr, "leaf_data is NULL");
    const int32_t L = (int32_t)n.sets.size();
    require(L == 1 || path_ssa != nullptr, "path is NULL");
    require(n_sliced >= 0 && n_sliced <= 255 && (n_sliced == 0 || sliced_ids),
            "bad slicing set (at most 255 indices)");
    auto p = new ltn_plan();
    std::unique_ptr<ltn_plan> guard(p);
    if (opt) p->opt = *opt;
    else p->opt.max_rank = -1;
    p->L = L;
    p->n_indices = n.n_indices;
    p->open_ids = n.open_ids;
    p->n_open = (int32_t)n.open_ids.size();
    require(p->n_open <= 62, "more than 62 open indices");
    // slicing set
    std::vector<int32_t> slice_bit(n.n_indices, -1);
    for (int32_t j = 0; j < n_sliced; ++j) {
      int32_t x = sliced_ids[j];
      require(x >= 0 && x < n.n_indices, "sliced id out of range");
      require(slice_bit[x] < 0, "sliced id " + std::to_string(x) + " listed twice");
      slice_bit[x] = j;
      p->sliced.push_back(x);
    }
    IdSet S(p->sliced.begin(), p->sliced.end());
    std::sort(S.begin(), S.end());
    // tree (validates the SSA cover)
    std::vector<int32_t> dummy;
    Tree tree = L > 1 ? Tree::build(n.sets, path_ssa) : Tree{};
    if (L == 1) {
      tree.L = 1;
      tree.sets = n.sets;
      tree.kids = {{-1, -1}};
      tree.parent = {-1};
    }
    const int32_t NT = (int32_t)tree.sets.size();
    p->root = NT - 1;
    // death step of every index
    const int32_t INF = INT32_MAX;
    std::vector<int32_t> death(n.n_indices, INF);
    for (int32_t k = 0; k + 1 < L; ++k) {
      auto [a, b] = tree.kids[L + k];
      for (int32_t x : set_and(tree.sets[a], tree.sets[b])) death[x] = k;
    }
    std::vector<int32_t> open_pos(n.n_indices, -1);
    for (int32_t j = 0; j < p->n_open; ++j) open_pos[n.open_ids[j]] = j;
    {
      IdSet rootset = tree.sets[p->root];
      IdSet opens(n.open_ids.begin(), n.open_ids.end());
      std::sort(opens.begin(), opens.end());
      require(rootset == opens, "the path does not end in a tensor holding exactly the open indices");
    }
    auto canon = [&](const IdSet& s) {
      IdSet u = set_minus(s, S);
      std::sort(u.begin(), u.end(), [&](int32_t x, int32_t y) {
        if (death[x] != death[y]) return death[x] < death[y];
        int32_t tx = death[x] == INF ? p->n_open - 1 - open_pos[x] : x;
        int32_t ty = death[y] == INF ? p->n_open - 1 - open_pos[y] : y;
        return tx < ty;
      });
      return u;
    };
    p->tensors.resize(NT);
    for (int32_t v = 0; v < NT; ++v) {
      TensorPlan& t = p->tensors[v];
      t.idx = canon(tree.sets[v]);
      t.rank = (int32_t)t.idx.size();
      if (p->opt.max_rank >= 0 && t.rank > p->opt.max_rank)
        fail(LTN_E_CAP, "tensor " + std::to_string(v) + " has rank " + std::to_string(t.rank) +
                            " after slicing, above max_rank " + std::to_string(p->opt.max_rank));
      require(t.rank <= 40, "tensor " + std::to_string(v) + " has rank " + std::to_string(t.rank) +
                                " after slicing; at most 40 is supported");
    }
    // steps
    int fat = p->opt.fat_threshold > 0 ? p->opt.fat_threshold : 4;
    for (int32_t k = 0; k + 1 < L; ++k) {
      StepPlan s;
      s.left = tree.kids[L + k].first;
      s.right = tree.kids[L + k].second;
      s.out = L + k;
      const IdSet& il = p->tensors[s.left].idx;
      const IdSet& ir = p->tensors[s.right].idx;
      s.a_is_left = il.size() >= ir.size() ? 1 : 0;
      s.a = s.a_is_left ? s.left : s.right;
      s.b = s.a_is_left ? s.right : s.left;
      const IdSet& A = p->tensors[s.a].idx;
      const IdSet& B = p->tensors[s.b].idx;
      int32_t kk = 0;
      while (kk < (int32_t)A.size() && death[A[kk]] == k) ++kk;
      int32_t kb = 0;
      while (kb < (int32_t)B.size() && death[B[kb]] == k) ++kb;
      require(kk == kb, "internal: operands disagree on contracted bits");
      for (int32_t j = 0; j < kk; ++j) require(A[j] == B[j], "internal: contracted bit order differs");
      s.k = kk;
      s.m = (int32_t)A.size() - kk;
      s.n = (int32_t)B.size() - kk;
      const IdSet& C = p->tensors[s.out].idx;
      require((int32_t)C.size() == s.m + s.n, "internal: output rank");
      int32_t ia = kk, ib = kk;
      for (int32_t j = 0; j < (int32_t)C.size(); ++j) {
        if (ia < (int32_t)A.size() && A[ia] == C[j]) {
          s.c_mask_a |= 1ull << j;
          ++ia;
        } else {
          require(ib < (int32_t)B.size() && B[ib] == C[j], "internal: output is not a merge");
          ++ib;
        }
      }
      s.kernel = (s.m >= fat + 1 && s.n >= fat && s.k >= fat - 1) ? LTN_K_MFMA : LTN_K_SMALL;
      p->tensors[s.a].consumer = k;
      p->tensors[s.b].consumer = k;
      p->tensors[s.out].producer = k;
      p->macs.add_pow2(s.m + s.k + s.n);
      p->steps.push_back(s);
    }
    p->macs_d = std::exp2(p->macs.log2());
    if (p->steps.empty()) p->macs_d = 0;
    // leaves: gather maps and data
    p->leaf_param = n.param;
    p->leaf_elems = n.data_off[L];
    p->leaf_data.assign(net->leaf_data, net->leaf_data + 2 * p->leaf_elems);
    for (int32_t i = 0; i < L; ++i) {
      LeafPlan lp;
      lp.leaf = i;
      lp.tensor = i;
      lp.src_off = n.data_off[i];
      lp.rank_src = (int32_t)n.axes[i].size();
      lp.rank = p->tensors[i].rank;
      lp.param = n.param[i];
      auto srcbit = [&](int32_t x) {
        for (int32_t q = 0; q < lp.rank_src; ++q)
          if (n.axes[i][q] == x) return lp.rank_src - 1 - q;
        return -1;
      };
      for (int32_t x : p->tensors[i].idx) lp.src_bit.push_back(srcbit(x));
      // sliced axes whose slice-id bit is 64 or above always take value 0
      for (int32_t x : n.axes[i])
        if (slice_bit[x] >= 0 && slice_bit[x] < 64) {
          lp.sl_src_bit.push_back(srcbit(x));
          lp.sl_bit.push_back(slice_bit[x]);
        }
      if (lp.param >= 0) {
        require(lp.rank_src == 2, "a parameterised leaf must have rank 2 (out, in)");
        p->n_params = std::max(p->n_params, 3 * (lp.param + 1));
      }
      p->leaves.push_back(lp);
    }
    // output placement
    {
      const IdSet& R = p->tensors[p->root].idx;
      for (int32_t x : R) p->out_mask |= 1ull << (p->n_open - 1 - open_pos[x]);
      for (int32_t j = 0; j < (int32_t)p->sliced.size() && j < 64; ++j) {
        int32_t x = p->sliced[j];
        if (open_pos[x] >= 0) p->out_sliced.push_back({j, p->n_open - 1 - open_pos[x]});
      }
    }
    // forward arena: leaves live from time 0, step k runs at time k+1, the
    // reduction at time L
    {
      std::vector<Block> live;
      uint64_t high = 0;
      auto t_end = [&](int32_t v) { return p->tensors[v].consumer >= 0 ? p->tensors[v].consumer + 1 : L; };
      for (int32_t v = 0; v < L; ++v)
        p->tensors[v].off = place_block(live, p->tensors[v].bytes(), 0, t_end(v), high);
      for (int32_t k = 0; k + 1 < L; ++k) {
        int32_t v = L + k;
        p->tensors[v].off = place_block(live, p->tensors[v].bytes(), k + 1, t_end(v), high);
      }
      p->arena = align_up(high, kAlign);
    }
    // split-precision steps read operand copies in the split layout
    for (auto& sp : p->steps)
      if (sp.kernel == LTN_K_MFMA && sp.k >= 3)
        p->split_scratch = std::max<uint64_t>(
            p->split_scratch, align_up(p->tensors[sp.a].bytes(), kAlign) + p->tensors[sp.b].bytes());
    p->split_scratch = align_up(p->split_scratch, kAlign);
    // grad arena: every tensor and its cotangent kept
    {
      uint64_t off = 0;
      for (auto& t : p->tensors) {
        off = align_up(off, std::min<uint64_t>(t.bytes(), kAlign));
        t.goff = off;
        off += t.bytes();
      }
      for (auto& t : p->tensors) {
        off = align_up(off, std::min<uint64_t>(t.bytes(), kAlign));
        t.gcot = off;
        off += t.bytes();
      }
      p->garena = align_up(off, kAlign);
    }
    *out = guard.release();
  });
}

extern "C" ltn_status ltn_plan_describe(const ltn_plan* p, ltn_plan_info* o) {
  return guarded([&] {
    require(p && o, "NULL argument");
    o->n_leaves = p->L;
    o->n_steps = (int32_t)p->steps.size();
    o->n_sliced = (int32_t)p->sliced.size();
    o->n_open = p->n_open;
    o->n_open_unsliced = p->tensors[p->root].rank;
    o->n_params = p->n_params;
    o->batch = 0;
    o->root_rank = p->tensors[p->root].rank;
    o->macs_per_slice = p->macs_d;
    p->macs.to_words(o->macs_words, 2);
    o->arena_bytes_per_slice = p->arena;
    o->grad_arena_bytes_per_slice = p->garena;
    o->const_bytes = 0;
    o->sliced_ids = p->sliced.data();
    runtime_describe(p, o);
  });
}

extern "C" ltn_status ltn_plan_step(const ltn_plan* p, int32_t step, ltn_step_info* o) {
  return guarded([&] {
    require(p && o, "NULL argument");
    require(step >= 0 && step < (int32_t)p->steps.size(), "step out of range");
    const StepPlan& s = p->steps[step];
    o->left = s.left;
    o->right = s.right;
    o->out = s.out;
    o->a_is_left = s.a_is_left;
    o->m = s.m;
    o->k = s.k;
    o->n = s.n;
    o->kernel = s.kernel;
    o->a_idx = p->tensors[s.a].idx.data();
    o->b_idx = p->tensors[s.b].idx.data();
    o->c_idx = p->tensors[s.out].idx.data();
    o->c_mask_a = s.c_mask_a;
    o->arena_off_a = p->tensors[s.a].off;
    o->arena_off_b = p->tensors[s.b].off;
    o->arena_off_c = p->tensors[s.out].off;
  });
}

extern "C" void ltn_plan_free(ltn_plan* p) {
  if (!p) return;
  runtime_free(p);
  delete p;
}
