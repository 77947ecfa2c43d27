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

namespace {

bool has(const IdSet& sorted, int32_t x) { return std::binary_search(sorted.begin(), sorted.end(), x); }

// The small operand Y of a step whose other operand is the chain tensor.
// Only steps of low arithmetic intensity are fused (rank(Y) = k + n <= 6):
// their cost is the HBM round trip that fusion removes; wider steps are
// better served by the matrix cores one step at a time.
bool small_other(const ltn_plan* p, const StepPlan& s, int32_t chain, int32_t* other) {
  int32_t y = s.a == chain ? s.b : (s.b == chain ? s.a : -1);
  if (y < 0) return false;
  const int32_t ry = p->tensors[y].rank, n = ry - s.k;
  if (ry > 6 || n > 6) return false;
  *other = y;
  return true;
}

// Build the group of the chain steps `steps` starting from tensor t0; false
// if a working tensor exceeds 2^R elements or the sub-path is unsuitable.
// Group of the chain steps `steps` from tensor t0 with the surviving
// indices `sig` (sorted) fixed per piece; false if unsuitable.
bool build_group(const ltn_plan* p, int32_t t0, const std::vector<int32_t>& steps, const IdSet& sig,
                 FuseGroup* g) {
  const int32_t tl = p->steps[steps.back()].out;
  const IdSet& I0 = p->tensors[t0].idx;
  const IdSet& IL = p->tensors[tl].idx;
  auto without = [&](const IdSet& v) {
    IdSet w;
    for (int32_t x : v)
      if (!has(sig, x)) w.push_back(x);
    return w;
  };
  FuseGroup G;
  G.t0 = t0;
  G.tl = tl;
  G.nsig = (int32_t)sig.size();
  G.a = (int32_t)I0.size() - G.nsig;
  // T_0's bits outside Sigma must be its lowest ones
  for (int32_t j = 0; j < G.a; ++j)
    if (has(sig, I0[j])) return false;
  IdSet w_prev = without(I0);
  G.rmax = (int32_t)w_prev.size();
  int32_t chain = t0;
  for (int32_t s : steps) {
    const StepPlan& sp = p->steps[s];
    int32_t y;
    if (!small_other(p, sp, chain, &y)) return false;
    const IdSet& Y = p->tensors[y].idx;
    FuseStage st;
    st.step = s;
    st.other = y;
    st.k = sp.k;
    st.n = (int32_t)Y.size() - sp.k;
    st.m = (int32_t)w_prev.size() - sp.k;
    if (st.m < 0) return false;
    for (int32_t j = 0; j < sp.k; ++j)
      if (w_prev[j] != Y[j]) return false;  // contracted bits lowest on both sides
    IdSet w_out = without(p->tensors[sp.out].idx);
    if ((int32_t)w_out.size() != st.m + st.n) return false;
    int32_t ia = sp.k;
    for (int32_t q = 0; q < (int32_t)w_out.size(); ++q)
      if (ia < (int32_t)w_prev.size() && w_prev[ia] == w_out[q]) {
        st.cmask |= 1ull << q;
        ++ia;
      }
    if (ia != (int32_t)w_prev.size()) return false;
    G.rmax = std::max<int32_t>(G.rmax, (int32_t)w_out.size());
    G.b_elems += 1 << p->tensors[y].rank;
    G.st.push_back(st);
    w_prev = w_out;
    chain = sp.out;
  }
  G.c = (int32_t)w_prev.size();
  for (int32_t q = 0; q < (int32_t)IL.size(); ++q) (has(sig, IL[q]) ? G.sig_out : G.w_out) |= 1ull << q;
  // Sigma keeps its relative order from T_0 to T_L
  {
    IdSet a0, aL;
    for (int32_t x : I0)
      if (has(sig, x)) a0.push_back(x);
    for (int32_t x : IL)
      if (has(sig, x)) aL.push_back(x);
    if (a0 != aL) return false;
  }
  if (G.b_elems > 2048 || (int)G.st.size() > kMaxFuseStages) return false;
  *g = G;
  return true;
}

// The indices of T_0 that survive to T_L, in T_0's bit order, are split:
// the first ones (those among T_L's lowest 4 bits, then more up to working
// rank R) are carried through every piece, the rest are fixed per piece.
// Carrying the earliest-contracted survivors keeps a piece's input one
// contiguous block of T_0 and makes its writes to T_L contiguous runs.
bool make_group(const ltn_plan* p, int32_t t0, const std::vector<int32_t>& steps, int R, FuseGroup* g) {
  const int32_t tl = p->steps[steps.back()].out;
  const IdSet& I0 = p->tensors[t0].idx;
  const IdSet& IL = p->tensors[tl].idx;
  IdSet sl(IL.begin(), IL.end());
  std::sort(sl.begin(), sl.end());
  std::vector<int32_t> surv;  // in T_0 order
  for (int32_t x : I0)
    if (has(sl, x)) surv.push_back(x);
  auto sig_after = [&](int q) {
    IdSet s(surv.begin() + q, surv.end());
    std::sort(s.begin(), s.end());
    return s;
  };
  int q0 = 0;
  for (int32_t q = 0; q < 4 && q < (int32_t)IL.size(); ++q)
    if (std::find(surv.begin(), surv.end(), IL[q]) != surv.end()) ++q0;
  FuseGroup G0;
  if (q0 > (int)surv.size() || !build_group(p, t0, steps, sig_after(q0), &G0) || G0.rmax > R) return false;
  const int extra = std::max(0, std::min(R - G0.rmax, (int)surv.size() - q0 - 3));
  if (extra == 0) {
    *g = G0;
    return true;
  }
  FuseGroup G1;
  if (!build_group(p, t0, steps, sig_after(q0 + extra), &G1) || G1.rmax > R) return false;
  *g = G1;
  return true;
}

// Greedy along the steps: start at a step whose larger operand has rank
// >= R + 3 and whose other operand is small, extend along the chain while
// the working tensors fit; keep sub-paths of at least two steps with
// |Sigma| >= 3 (at least 8 pieces per slice).
void find_groups(ltn_plan* p, int R) {
  const int32_t ns = (int32_t)p->steps.size();
  for (int32_t s = 0; s < ns; ++s) {
    if (p->step_group[s] >= 0) continue;
    const StepPlan& sp = p->steps[s];
    const int32_t t0 = sp.a;
    int32_t y;
    if (p->tensors[t0].rank < R + 3 || !small_other(p, sp, t0, &y)) continue;
    std::vector<int32_t> steps{s};
    FuseGroup best;
    bool have = false;
    for (;;) {
      FuseGroup g;
      if (!make_group(p, t0, steps, R, &g)) break;
      if (steps.size() >= 2 && g.nsig >= 3) {
        best = g;
        have = true;
      }
      const int32_t nxt = p->tensors[p->steps[steps.back()].out].consumer;
      if (nxt < 0 || p->step_group[nxt] >= 0) break;
      steps.push_back(nxt);
    }
    if (!have) continue;
    for (auto& st : best.st) p->step_group[st.step] = (int32_t)p->groups.size();
    p->groups.push_back(best);
  }
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
    // fused sub-paths (secondary slicing, Sec. 5.2)
    p->step_group.assign(p->steps.size(), -1);
    std::vector<int32_t> keep_until(NT, -1);  // extended lifetimes (step index)
    if (p->opt.fuse_rank > 0) {
      require(p->opt.fuse_rank <= 11, "fuse_rank must be at most 11");
      find_groups(p, p->opt.fuse_rank);
      for (auto& g : p->groups) {
        const int32_t last = g.st.back().step;
        keep_until[g.t0] = last;
        for (auto& s : g.st) keep_until[s.other] = last;
      }
    }
    // forward arena: leaves live from time 0, step k runs at time k+1, the
    // reduction at time L; a fused sub-path runs at its last step, so T_0
    // and the small tensors stay live until then
    {
      std::vector<Block> live;
      uint64_t high = 0;
      auto t_end = [&](int32_t v) {
        int32_t e = p->tensors[v].consumer >= 0 ? p->tensors[v].consumer + 1 : L;
        return std::max(e, keep_until[v] + 1);
      };
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

extern "C" ltn_status ltn_plan_groups(const ltn_plan* p, int32_t* first_step, int32_t* n_steps,
                                     int32_t* n_sigma, int32_t* work_rank, int32_t cap, int32_t* n) {
  return guarded([&] {
    require(p && n, "NULL argument");
    require((int32_t)p->groups.size() <= cap || p->groups.empty(), "arrays too small", LTN_E_NOMEM);
    for (size_t g = 0; g < p->groups.size(); ++g) {
      if (first_step) first_step[g] = p->groups[g].st.front().step;
      if (n_steps) n_steps[g] = (int32_t)p->groups[g].st.size();
      if (n_sigma) n_sigma[g] = p->groups[g].nsig;
      if (work_rank) work_rank[g] = p->groups[g].rmax;
    }
    *n = (int32_t)p->groups.size();
  });
}
