// Device side of a plan: workspace layout, batch execution (leaf gather ->
// contraction steps -> FP64 slice sum), hipGraph capture and replay, the
// adjoint sweep for gradients, tile autotuning and per-step profiling.
//
// Everything runs on the stream given to ltn_bind; the library allocates no
// device memory of its own (the caller's workspace holds leaf data,
// descriptors, slice ids, the per-slice arenas and gradient accumulators).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "kernels.h"
#include "plan.h"

using namespace ltn;

#define HIPCHECK(x)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      fail(LTN_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_) + " (" +         \
                          std::to_string((int)e_) + ")");                               \
  } while (0)

struct Layout {
  size_t leafdata, gd_fwd, gd_grad, gd_gcot, pl, angles, leafgrad, ids, scales, arena, split, gscr,
      gscr_c, skinny, splitk, gdesc, fdesc, total;
};

struct ltn_plan_impl {
  hipStream_t st = nullptr;
  hipStream_t cap = nullptr;  // capture stream (the null stream cannot be captured)
  char* ws = nullptr;
  size_t bytes = 0;
  int grad = 0;
  int B = 0;
  Layout lay{};
  int n_pl = 0;
  int max_leaf_elems = 1;
  int64_t gather_chunks = 0;  // blocks per slice of the leaf gather
  std::vector<GatherDesc> gd_fwd, gd_grad, gd_gcot;
  std::vector<ParamLeaf> pl;
  std::vector<int32_t> sl_bits, out_bits;
  bool fuse = true;  // run fused sub-paths in forward passes
  // kernel choice per mode and step: kind 0 = generic (tk threads per
  // output), 1 = complex64 MFMA GEMM, 2 = split MFMA GEMM (cfg, swap),
  // 3 = narrow-step kernel (swap: rows taken from the B operand), 4 = split
  // sum over k for steps with few outputs, 5 = split-K complex64 MFMA GEMM
  // (cfg, swap) for long sums with too few columns for a full tile
  struct Choice {
    int kind = 0, cfg = -1, swap = 0, tk = 1;
  };
  std::vector<Choice> choice[3];
  // adjoint products (forward-form GEMMs of the gradient sweep) by shape
  // (m | k << 8 | n << 16): kind 1 = a complex64 tile, kind 5 = a split-K
  // tile (cfg, swap) chosen by ltn_autotune; absent = the fixed rule of
  // enqueue_nt
  std::map<uint32_t, Choice> adj;
  std::vector<char> needs_grad;
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
  hipGraph_t graph_src[3] = {nullptr, nullptr, nullptr};
  // gradients, full batches: recomputed forward and adjoint sweep
  hipGraphExec_t ggraph[2] = {nullptr, nullptr};
  hipGraph_t ggraph_src[2] = {nullptr, nullptr};
  // gradient launch sequence: runs of independent generic contractions of
  // consecutive steps share one launch (descriptors in the workspace)
  struct GradItem {
    int what = 0;  // 0: forward step, 1: generic run, 2: large adjoint step
    int step = -1, off = 0, count = 0, tk = 1;
    uint64_t max_outs = 0;
  };
  // forward kept in the gradient arena by the last ltn_execute (plan bound
  // for gradients, complex64, one batch) and its slice ids: ltn_execute_grad
  // on the same ids skips recomputing it; ltn_set_params and every other use
  // of the arena drop it
  bool fwd_kept = false;
  std::vector<uint64_t> fwd_ids;
  bool gseq_valid = false;
  std::vector<GenericDesc> gseq_descs;
  std::vector<GradItem> gseq_fwd, gseq_bwd;
  // forward launch sequence per mode (what 0: step, 1: generic run, 3: fused group)
  bool fseq_valid[3] = {false, false, false};
  std::vector<GenericDesc> fseq_descs[3];
  std::vector<GradItem> fseq[3];
  std::vector<uint64_t> host_ids;
};

namespace {

size_t al(size_t x) { return (x + 255) / 256 * 256; }

Layout layout(const ltn_plan* p, int B, int grad) {
  Layout l{};
  size_t o = 0;
  int npl = 0;
  for (auto& lp : p->leaves) npl += lp.param >= 0;
  l.leafdata = o;
  o = al(o + (size_t)p->leaf_elems * 8);
  l.gd_fwd = o;
  o = al(o + p->leaves.size() * sizeof(GatherDesc));
  l.gd_grad = o;
  o = al(o + (grad ? p->leaves.size() * sizeof(GatherDesc) : 0));
  l.gd_gcot = o;
  o = al(o + (grad ? p->leaves.size() * sizeof(GatherDesc) : 0));
  l.pl = o;
  o = al(o + (size_t)npl * sizeof(ParamLeaf));
  l.angles = o;
  o = al(o + (size_t)p->n_params * sizeof(double));
  l.leafgrad = o;
  o = al(o + (size_t)npl * 8 * sizeof(double));
  l.ids = o;
  o = al(o + (size_t)B * 8);
  l.scales = o;  // per tensor and slice: max |Re|, |Im|; then split_f16 bounds
  o = al(o + (size_t)B * p->tensors.size() * 8);
  l.arena = o;
  o = al(o + (size_t)B * (grad ? p->garena : p->arena));
  l.split = o;
  o = al(o + (size_t)B * p->split_scratch);
  // adjoint scratch: a permuted copy of an output cotangent and of one operand
  size_t sc = 0, so = 0;
  if (grad)
    for (auto& sp : p->steps) {
      sc = std::max<size_t>(sc, p->tensors[sp.out].bytes());
      so = std::max<size_t>(so, std::max(p->tensors[sp.a].bytes(), p->tensors[sp.b].bytes()));
    }
  l.gscr = o;
  o = al(o + (size_t)B * so);
  l.gscr_c = o;
  o = al(o + (size_t)B * sc);
  // partial sums of the few-output steps (largest over the steps that fit)
  int64_t sk = 0;
  for (auto& sp : p->steps)
    if (skinny_fits(sp.m, sp.k, sp.n)) sk = std::max<int64_t>(sk, skinny_part_elems(sp.m, sp.k, sp.n));
  l.skinny = o;
  o = al(o + (size_t)B * (size_t)sk * 8);
  // split-K partials (largest over the steps a split-K tile fits and, on
  // plans bound for gradients, over the adjoint products)
  int64_t kp = 0;
  for (auto& sp : p->steps) {
    kp = std::max<int64_t>(kp, splitk_part_elems(sp.m, sp.k, sp.n));
    if (grad) {
      kp = std::max<int64_t>(kp, splitk_part_elems(sp.m, sp.n, sp.k));
      kp = std::max<int64_t>(kp, splitk_part_elems(sp.n, sp.m, sp.k));
    }
  }
  l.splitk = o;
  o = al(o + (size_t)B * (size_t)kp * 8);
  l.gdesc = o;  // gradient runs: at most one descriptor per step forward, two backward
  if (grad) o = al(o + 3 * p->steps.size() * sizeof(GenericDesc));
  l.fdesc = o;  // forward runs: one descriptor per step and mode
  o = al(o + 3 * std::max<size_t>(1, p->steps.size()) * sizeof(GenericDesc));
  l.total = o;
  return l;
}

ltn_plan_impl& rt(ltn_plan* p) {
  if (!p || !p->rt || !p->rt->ws) fail(LTN_E_STATE, "plan is not bound (call ltn_bind first)");
  return *p->rt;
}

float2* arena_ptr(ltn_plan* p, uint64_t off_bytes) {
  auto& r = *p->rt;
  return reinterpret_cast<float2*>(r.ws + r.lay.arena + off_bytes * (uint64_t)r.B);
}

// Untuned complex64 tiles: the three-product tiles first, then the direct
// tiles 0-7 (sums shorter than 16); split modes: in order.
int default_cfg(int m, int k, int n, int mode) {
  static const int c64_order[] = {10, 15, 13, 0, 1, 2, 3, 4, 5, 6, 7};
  if (mode == LTN_C64) {
    for (int c : c64_order)
      if (gemm_config_fits(c, m, k, n, mode)) return c;
    return -1;
  }
  for (int c = 0; c < gemm_config_count(mode); ++c)
    if (gemm_config_fits(c, m, k, n, mode)) return c;
  return -1;
}

int default_tk(int k, uint64_t outs) {
  int tk = k <= 3 ? 1 : (k <= 6 ? 8 : 64);
  if (outs < (1u << 16) && k >= 3) tk = std::max(tk, 8);
  if (outs < (1u << 12) && k >= 5) tk = 64;
  return tk;
}

uint32_t* slot(ltn_plan* p, int tensor) {
  auto& r = *p->rt;
  return reinterpret_cast<uint32_t*>(r.ws + r.lay.scales) + (size_t)tensor * r.B;
}

// split_f16: the bound whose scale a producer used to write the tensor in
// the split layout (read by the consumer in place of the tensor's maximum)
uint32_t* bound_slot(ltn_plan* p, int tensor) {
  return slot(p, (int)p->tensors.size() + tensor);
}

// Split modes: a tensor that a matrix-core step produces and a split step
// consumes is written by its producer in the split layout, and the
// conversion pass before the consumer is skipped. bf16 needs no scale; for
// fp16 the producer cannot know its output's maximum before writing, so it
// scales by the bound 2 K max|a| max|b| taken from its operands' recorded
// maxima (stored for the consumer). Steps run inside a fused sub-path read
// and write complex64, and the gradient's recomputed forward stays complex64.
bool split_direct(ltn_plan* p, int t, int mode, bool gradarena) {
  if (mode == LTN_C64 || gradarena) return false;
  auto& r = *p->rt;
  const TensorPlan& T = p->tensors[t];
  if (T.producer < 0 || T.consumer < 0) return false;
  auto fused = [&](int s) { return r.fuse && p->step_group[s] >= 0; };
  if (fused(T.producer) || fused(T.consumer)) return false;
  const int kp = r.choice[mode][T.producer].kind, kc = r.choice[mode][T.consumer].kind;
  return (kp == 1 || kp == 2) && kc == 2;
}

// The generic kernel's descriptor for forward step s.
GenericDesc step_generic_desc(ltn_plan* p, int s, int nb, bool gradarena, int mode) {
  const StepPlan& sp = p->steps[s];
  const TensorPlan &ta = p->tensors[sp.a], &tb = p->tensors[sp.b], &tc = p->tensors[sp.out];
  const uint64_t cm = sp.c_mask_a, full = (sp.m + sp.n) >= 64 ? ~0ull : ((1ull << (sp.m + sp.n)) - 1);
  GenericDesc g{};
  g.P = arena_ptr(p, gradarena ? ta.goff : ta.off);
  g.Q = arena_ptr(p, gradarena ? tb.goff : tb.off);
  g.out = arena_ptr(p, gradarena ? tc.goff : tc.off);
  g.sP = int64_t(1) << ta.rank;
  g.sQ = int64_t(1) << tb.rank;
  g.sO = int64_t(1) << tc.rank;
  g.xb = sp.m;
  g.yb = sp.n;
  g.zb = sp.k;
  g.px = ((1ull << sp.m) - 1) << sp.k;
  g.pz = (1ull << sp.k) - 1;
  g.qy = ((1ull << sp.n) - 1) << sp.k;
  g.qz = (1ull << sp.k) - 1;
  g.ox = cm;
  g.oy = ~cm & full;
  g.nb = nb;
  if (mode == LTN_SPLIT_F16) g.scale_out = slot(p, sp.out);
  return g;
}

void enqueue_step(ltn_plan* p, int s, int nb, bool gradarena, int mode) {
  auto& r = *p->rt;
  const StepPlan& sp = p->steps[s];
  const TensorPlan &ta = p->tensors[sp.a], &tb = p->tensors[sp.b], &tc = p->tensors[sp.out];
  float2* A = arena_ptr(p, gradarena ? ta.goff : ta.off);
  float2* B = arena_ptr(p, gradarena ? tb.goff : tb.off);
  float2* C = arena_ptr(p, gradarena ? tc.goff : tc.off);
  const uint64_t cm = sp.c_mask_a, full = (sp.m + sp.n) >= 64 ? ~0ull : ((1ull << (sp.m + sp.n)) - 1);
  const auto& ch = r.choice[mode][s];
  const bool split = mode != LTN_C64;
  if (ch.kind == 4) {
    SkinnyDesc d{};
    d.A = A;
    d.B = B;
    d.C = C;
    d.sA = int64_t(1) << ta.rank;
    d.sB = int64_t(1) << tb.rank;
    d.sC = int64_t(1) << tc.rank;
    d.m = sp.m;
    d.k = sp.k;
    d.n = sp.n;
    d.cmask = cm;
    d.nb = nb;
    d.part = reinterpret_cast<float2*>(r.ws + r.lay.skinny);
    if (mode == LTN_SPLIT_F16) d.scale_c = slot(p, sp.out);
    launch_skinny(d, r.st);
    return;
  }
  if (ch.kind == 5) {
    GemmDesc d{};
    const bool sw = ch.swap;
    d.A = sw ? B : A;
    d.B = sw ? A : B;
    d.C = C;
    d.sA = int64_t(1) << (sw ? tb.rank : ta.rank);
    d.sB = int64_t(1) << (sw ? ta.rank : tb.rank);
    d.sC = int64_t(1) << tc.rank;
    d.m = sw ? sp.n : sp.m;
    d.n = sw ? sp.m : sp.n;
    d.k = sp.k;
    d.cmask = sw ? (~cm & full) : cm;
    d.nb = nb;
    d.cfg = ch.cfg;
    d.part = reinterpret_cast<float2*>(r.ws + r.lay.splitk);
    if (mode == LTN_SPLIT_F16) d.scale_c = slot(p, sp.out);
    launch_cgemm_splitk(d, r.st);
    return;
  }
  if (ch.kind == 3) {
    NarrowDesc d{};
    const bool sw = ch.swap;
    d.A = sw ? B : A;
    d.B = sw ? A : B;
    d.C = C;
    d.sA = int64_t(1) << (sw ? tb.rank : ta.rank);
    d.sB = int64_t(1) << (sw ? ta.rank : tb.rank);
    d.sC = int64_t(1) << tc.rank;
    d.m = sw ? sp.n : sp.m;
    d.n = sw ? sp.m : sp.n;
    d.k = sp.k;
    d.cmask = sw ? (~cm & full) : cm;
    d.nb = nb;
    d.cfg = ch.cfg;
    if (mode == LTN_SPLIT_F16) d.scale_c = slot(p, sp.out);
    launch_narrow(d, r.st);
    return;
  }
  if (ch.kind > 0) {
    GemmDesc d{};
    bool sw = ch.swap;
    d.A = sw ? B : A;
    d.B = sw ? A : B;
    d.C = C;
    d.sA = int64_t(1) << (sw ? tb.rank : ta.rank);
    d.sB = int64_t(1) << (sw ? ta.rank : tb.rank);
    d.sC = int64_t(1) << tc.rank;
    d.m = sw ? sp.n : sp.m;
    d.n = sw ? sp.m : sp.n;
    d.k = sp.k;
    d.cmask = sw ? (~cm & full) : cm;
    d.nb = nb;
    d.cfg = ch.cfg;
    const bool f16 = mode == LTN_SPLIT_F16;
    if (f16) d.scale_c = slot(p, sp.out);
    if (split_direct(p, sp.out, mode, gradarena)) {
      d.split_out = f16 ? 2 : 1;
      if (f16) {
        d.max_a = slot(p, sw ? sp.b : sp.a);
        d.max_b = slot(p, sw ? sp.a : sp.b);
        d.bound_c = bound_slot(p, sp.out);
      }
    }
    if (ch.kind == 2) {
      // split-layout copies of both operands in the per-batch scratch area,
      // unless the producer wrote them so
      float2* As = reinterpret_cast<float2*>(r.ws + r.lay.split);
      float2* Bs = As + (((ta.bytes() + 255) / 256 * 256) / 8) * (uint64_t)r.B;
      if (split_direct(p, sp.a, mode, gradarena))
        As = A;
      else
        launch_split_convert(A, As, ta.rank, nb, f16 ? slot(p, sp.a) : nullptr, mode, r.st);
      if (split_direct(p, sp.b, mode, gradarena))
        Bs = B;
      else
        launch_split_convert(B, Bs, tb.rank, nb, f16 ? slot(p, sp.b) : nullptr, mode, r.st);
      d.A = sw ? Bs : As;
      d.B = sw ? As : Bs;
      if (f16) {
        // the maximum the operand's split copy was scaled by, or the bound
        // its producer used
        const int ra = sw ? sp.b : sp.a, rb = sw ? sp.a : sp.b;
        d.scale_a = split_direct(p, ra, mode, gradarena) ? bound_slot(p, ra) : slot(p, ra);
        d.scale_b = split_direct(p, rb, mode, gradarena) ? bound_slot(p, rb) : slot(p, rb);
      }
    }
    launch_cgemm(d, ch.kind == 2 ? mode : LTN_C64, r.st);
  } else {
    GenericDesc g = step_generic_desc(p, s, nb, gradarena, mode);
    launch_generic(g, ch.tk, r.st);
  }
}

// A fused sub-path at its last step (the plan keeps T_0 and the small
// tensors live until then).
void enqueue_group(ltn_plan* p, int g, int nb, int mode) {
  auto& r = *p->rt;
  const FuseGroup& G = p->groups[g];
  FusedDesc d{};
  d.X0 = arena_ptr(p, p->tensors[G.t0].off);
  d.XL = arena_ptr(p, p->tensors[G.tl].off);
  d.sX0 = int64_t(1) << p->tensors[G.t0].rank;
  d.sXL = int64_t(1) << p->tensors[G.tl].rank;
  d.a = G.a;
  d.nsig = G.nsig;
  d.c = G.c;
  d.rmax = G.rmax;
  d.nstages = (int32_t)G.st.size();
  d.nb = nb;
  d.sig_out = G.sig_out;
  d.w_out = G.w_out;
  if (mode == LTN_SPLIT_F16) d.scale_c = slot(p, G.tl);
  int yoff = 0;
  for (int j = 0; j < d.nstages; ++j) {
    const FuseStage& s = G.st[j];
    FusedStage& f = d.st[j];
    f.Y = arena_ptr(p, p->tensors[s.other].off);
    f.sY = int64_t(1) << p->tensors[s.other].rank;
    f.m = s.m;
    f.k = s.k;
    f.n = s.n;
    f.cmask = s.cmask;
    f.yoff = yoff;
    yoff += 1 << (s.k + s.n);
  }
  d.y_elems = yoff;
  launch_fused(d, r.st);
}

void enqueue_forward(ltn_plan* p, int nb, bool gradarena, int mode) {
  auto& r = *p->rt;
  const GatherDesc* gd = reinterpret_cast<const GatherDesc*>(r.ws + (gradarena ? r.lay.gd_grad : r.lay.gd_fwd));
  uint32_t* scales = nullptr;
  if (mode == LTN_SPLIT_F16) {
    scales = reinterpret_cast<uint32_t*>(r.ws + r.lay.scales);
    launch_fill_zero(scales, al((size_t)r.B * p->tensors.size() * 4), r.st);
  }
  launch_gather(gd, (int)p->leaves.size(), r.gather_chunks, r.max_leaf_elems,
                reinterpret_cast<const float2*>(r.ws + r.lay.leafdata), arena_ptr(p, 0),
                reinterpret_cast<const uint64_t*>(r.ws + r.lay.ids), nb, scales, r.B, r.st);
  if (gradarena && r.gseq_valid) {
    const GenericDesc* dd = reinterpret_cast<const GenericDesc*>(r.ws + r.lay.gdesc);
    for (const auto& it : r.gseq_fwd) {
      if (it.what == 0)
        enqueue_step(p, it.step, nb, true, mode);
      else
        launch_generic_multi(dd + it.off, it.count, it.max_outs, nb, it.tk, r.st);
    }
    return;
  }
  if (!gradarena && r.fseq_valid[mode]) {
    const GenericDesc* dd =
        reinterpret_cast<const GenericDesc*>(r.ws + r.lay.fdesc) + (size_t)mode * p->steps.size();
    for (const auto& it : r.fseq[mode]) {
      if (it.what == 0)
        enqueue_step(p, it.step, nb, false, mode);
      else if (it.what == 3)
        enqueue_group(p, it.step, nb, mode);
      else
        launch_generic_multi(dd + it.off, it.count, it.max_outs, nb, it.tk, r.st);
    }
    return;
  }
  for (int s = 0; s < (int)p->steps.size(); ++s) {
    const int g = p->step_group[s];
    if (g >= 0 && r.fuse && !gradarena) {
      if (s == p->groups[g].st.back().step) enqueue_group(p, g, nb, mode);
      continue;
    }
    enqueue_step(p, s, nb, gradarena, mode);
  }
}

// Forward launch sequence of a mode: consecutive generic steps share one
// launch unless one of them reads, or writes over, memory another one
// writes or reads (the arena reuses memory once a tensor is dead, so the
// test is on per-slice byte ranges, not tensor ids). Fused sub-paths keep
// their launch at their last step. Descriptors (for the bound batch size)
// are copied to the workspace here, outside any capture.
void build_fwd_seq(ltn_plan* p, int mode) {
  auto& r = *p->rt;
  using Item = ltn_plan_impl::GradItem;
  auto& seq = r.fseq[mode];
  auto& descs = r.fseq_descs[mode];
  seq.clear();
  descs.clear();
  struct Range {
    uint64_t lo, hi;
  };
  auto range = [&](int t) { return Range{p->tensors[t].off, p->tensors[t].off + p->tensors[t].bytes()}; };
  auto overlap = [](Range a, Range b) { return a.lo < b.hi && b.lo < a.hi; };
  std::vector<std::pair<GenericDesc, int>> run;
  std::vector<Range> reads, writes;
  auto flush = [&]() {
    for (int tk : {1, 8, 64}) {
      Item it;
      it.what = 1;
      it.tk = tk;
      it.off = (int)descs.size();
      for (auto& e : run)
        if (e.second == tk) {
          descs.push_back(e.first);
          it.max_outs = std::max<uint64_t>(it.max_outs, 1ull << (e.first.xb + e.first.yb));
        }
      it.count = (int)descs.size() - it.off;
      if (it.count) seq.push_back(it);
    }
    run.clear();
    reads.clear();
    writes.clear();
  };
  for (int s = 0; s < (int)p->steps.size(); ++s) {
    const StepPlan& sp = p->steps[s];
    const int g = p->step_group[s];
    if (g >= 0 && r.fuse) {
      if (s == p->groups[g].st.back().step) {
        flush();
        Item it;
        it.what = 3;
        it.step = g;
        seq.push_back(it);
      }
      continue;
    }
    const auto& ch = r.choice[mode][s];
    if (ch.kind != 0) {
      flush();
      Item it;
      it.what = 0;
      it.step = s;
      seq.push_back(it);
      continue;
    }
    const Range ra = range(sp.a), rb = range(sp.b), rc = range(sp.out);
    bool clash = false;
    for (auto& w : writes) clash = clash || overlap(w, ra) || overlap(w, rb) || overlap(w, rc);
    for (auto& q : reads) clash = clash || overlap(q, rc);
    if (clash) flush();
    run.push_back({step_generic_desc(p, s, r.B, false, mode), ch.tk});
    reads.push_back(ra);
    reads.push_back(rb);
    writes.push_back(rc);
  }
  flush();
  require(descs.size() <= p->steps.size(), "forward descriptor area too small");
  if (!descs.empty()) {
    char* dst = r.ws + r.lay.fdesc + (size_t)mode * p->steps.size() * sizeof(GenericDesc);
    HIPCHECK(hipMemcpyAsync(dst, descs.data(), descs.size() * sizeof(GenericDesc), hipMemcpyHostToDevice, r.st));
    // the host array may be rebuilt by a later call: let the copy finish
    HIPCHECK(hipStreamSynchronize(r.st));
  }
  r.fseq_valid[mode] = true;
}

void enqueue_reduce(ltn_plan* p, int nb, bool gradarena, double* out) {
  auto& r = *p->rt;
  const TensorPlan& root = p->tensors[p->root];
  launch_reduce(arena_ptr(p, gradarena ? root.goff : root.off), root.rank, p->out_mask,
                r.sl_bits.data(), r.out_bits.data(), (int)r.sl_bits.size(),
                reinterpret_cast<const uint64_t*>(r.ws + r.lay.ids), nb, out, r.st);
}

void set_ids(ltn_plan* p, const uint64_t* ids, uint64_t base, int n, bool range) {
  auto& r = *p->rt;
  uint64_t* d = reinterpret_cast<uint64_t*>(r.ws + r.lay.ids);
  if (range)
    launch_set_range(d, base, n, r.st);
  else
    launch_set_ids(d, ids, n, r.st);
}

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(LTN_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

// Launch the work `enqueue` issues as one graph on the bound stream,
// capturing it (on a stream of our own) the first time. The captured
// kernels keep their arguments, so only work whose pointers and shapes are
// fixed for the bound workspace goes in.
template <typename F>
void launch_captured(ltn_plan* p, hipGraphExec_t& exec, hipGraph_t& src, F&& enqueue) {
  auto& r = *p->rt;
  if (!exec) {
    if (!r.cap) HIPCHECK(hipStreamCreateWithFlags(&r.cap, hipStreamNonBlocking));
    hipGraph_t g;
    hipStream_t bound = r.st;
    r.st = r.cap;
    hipError_t e = hipStreamBeginCapture(r.cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        enqueue();
      } catch (...) {
        r.st = bound;
        (void)hipStreamEndCapture(r.cap, &g);
        throw;
      }
      e = hipStreamEndCapture(r.cap, &g);
    }
    r.st = bound;
    if (e != hipSuccess) fail(LTN_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    HIPCHECK(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
    src = g;
  }
  HIPCHECK(hipGraphLaunch(exec, r.st));
}

void run_batch(ltn_plan* p, int nb, int mode, double* out) {
  auto& r = *p->rt;
  if (!r.fseq_valid[mode]) build_fwd_seq(p, mode);
  if (nb == r.B) {
    launch_captured(p, r.graph[mode], r.graph_src[mode], [&] { enqueue_forward(p, nb, false, mode); });
  } else {
    enqueue_forward(p, nb, false, mode);
  }
  enqueue_reduce(p, nb, false, out);
  check_launch();
}

void check_mode(int mode) {
  require(mode == LTN_C64 || mode == LTN_SPLIT_F16 || mode == LTN_SPLIT_BF16, "unknown mode");
}

}  // namespace

void runtime_describe(const ltn_plan* p, ltn_plan_info* o) {
  if (p->rt) o->batch = p->rt->B;
  o->const_bytes = layout(p, 0, 0).total;
}

void runtime_free(ltn_plan* p) {
  if (!p->rt) return;
  for (int m = 0; m < 3; ++m) {
    if (p->rt->graph[m]) (void)hipGraphExecDestroy(p->rt->graph[m]);
    if (p->rt->graph_src[m]) (void)hipGraphDestroy(p->rt->graph_src[m]);
  }
  for (int m = 0; m < 2; ++m) {
    if (p->rt->ggraph[m]) (void)hipGraphExecDestroy(p->rt->ggraph[m]);
    if (p->rt->ggraph_src[m]) (void)hipGraphDestroy(p->rt->ggraph_src[m]);
  }
  if (p->rt->cap) (void)hipStreamDestroy(p->rt->cap);
  delete p->rt;
  p->rt = nullptr;
}

extern "C" ltn_status ltn_workspace_size(const ltn_plan* p, int32_t batch, int32_t grad,
                                         size_t* bytes) {
  return guarded([&] {
    require(p && bytes, "NULL argument");
    require(batch >= 1, "batch must be >= 1");
    *bytes = layout(p, batch, grad).total;
  });
}

namespace {

// Largest batch whose workspace fits in `bytes`, at most `cap` (0 when not
// even one slice fits).
int fit_batch(const ltn_plan* p, size_t bytes, int grad, int cap) {
  int B = std::min(p->opt.batch > 0 ? p->opt.batch : 4096, 4096);
  if (p->sliced.size() < 12) B = std::min(B, 1 << p->sliced.size());
  B = std::max(1, std::min(B, cap));
  while (B > 1 && layout(p, B, grad).total > bytes) {
    size_t per = grad ? p->garena : p->arena;
    size_t fixed = layout(p, 0, grad).total;
    size_t fit = bytes > fixed ? (bytes - fixed) / (per + 8 + 4 * p->tensors.size() + 512) : 0;
    B = (int)std::max<size_t>(1, std::min<size_t>(fit, (size_t)B - 1));
    if (layout(p, B, grad).total <= bytes) break;
  }
  return layout(p, B, grad).total <= bytes ? B : 0;
}

// Fill a device-side state for the workspace d_ws (batch B): gather
// descriptors, default kernel choices, and the uploads of leaf data and
// descriptors, synchronised on `st` before returning.
void bind_state(ltn_plan* p, ltn_plan_impl* r, char* d_ws, size_t bytes, int grad, hipStream_t st,
                int B) {
  r->st = st;
  r->ws = d_ws;
  r->bytes = bytes;
  r->grad = grad;
  r->B = B;
  r->lay = layout(p, B, grad);
  // descriptors
  int gi = 0;
  for (auto& lp : p->leaves) {
    require(lp.rank_src <= kMaxLeafRank, "leaf rank above 32 is not supported");
    GatherDesc g{};
    g.src_off = lp.src_off;
    g.chunk0 = r->gather_chunks;
    r->gather_chunks += ((int64_t(1) << lp.rank) + kGatherChunk - 1) / kGatherChunk;
    g.rank = lp.rank;
    g.nsl = (int32_t)lp.sl_bit.size();
    for (int j = 0; j < lp.rank; ++j) g.src_bit[j] = (int8_t)lp.src_bit[j];
    for (int j = 0; j < g.nsl; ++j) {
      g.sl_src_bit[j] = (int8_t)lp.sl_src_bit[j];
      g.sl_bit[j] = (int8_t)lp.sl_bit[j];
    }
    const TensorPlan& t = p->tensors[lp.tensor];
    g.tensor = lp.tensor;
    g.dst_off = (int64_t)(t.off * (uint64_t)B / 8);
    r->gd_fwd.push_back(g);
    g.dst_off = (int64_t)(t.goff * (uint64_t)B / 8);
    r->gd_grad.push_back(g);
    g.dst_off = (int64_t)(t.gcot * (uint64_t)B / 8);
    r->gd_gcot.push_back(g);
    r->max_leaf_elems = lp.rank >= 30 ? (1 << 30) : std::max(r->max_leaf_elems, 1 << lp.rank);
    if (lp.param >= 0) r->pl.push_back(ParamLeaf{lp.src_off, lp.param, gi});
    ++gi;
  }
  r->n_pl = (int)r->pl.size();
  for (auto& pr : p->out_sliced) {
    r->sl_bits.push_back(pr.first);
    r->out_bits.push_back(pr.second);
  }
  require(r->sl_bits.size() <= 32, "more than 32 sliced open indices");
  // kernel choice per mode and step (refined by ltn_autotune)
  for (int mode = 0; mode < 3; ++mode)
    for (auto& sp : p->steps) {
      ltn_plan_impl::Choice ch;
      ch.tk = default_tk(sp.k, (1ull << (sp.m + sp.n)) * (uint64_t)B);
      if (sp.kernel == LTN_K_MFMA) {
        // MFMA columns follow the output's lowest bits when possible
        bool nat = (sp.c_mask_a & 1) != 0;
        for (int kind : {mode == LTN_C64 ? 1 : 2, 1}) {
          int km = kind == 2 ? mode : LTN_C64;
          for (bool sw : {nat, !nat}) {
            int c = sw ? default_cfg(sp.n, sp.k, sp.m, km) : default_cfg(sp.m, sp.k, sp.n, km);
            if (c >= 0 && ch.kind == 0) {
              ch.kind = kind;
              ch.cfg = c;
              ch.swap = sw;
            }
          }
        }
      }
      // no full tile but a long sum: the split-K tile (the small side as columns)
      if (ch.kind == 0) {
        const bool sw = sp.n > sp.m;
        for (int c = 0; c < splitk_config_count() && ch.kind == 0; ++c)
          if (sw ? splitk_config_fits(c, sp.n, sp.k, sp.m) : splitk_config_fits(c, sp.m, sp.k, sp.n)) {
            ch.kind = 5;
            ch.cfg = c;
            ch.swap = sw;
          }
      }
      // few outputs and a long sum: split the sum over blocks
      if (ch.kind == 0 && skinny_fits(sp.m, sp.k, sp.n) && sp.k >= 10) {
        ch.kind = 4;
        ch.cfg = 0;
      }
      // steps with many output rows and no MFMA tile: the narrow kernel
      if (ch.kind == 0 && sp.m + sp.n >= 12) {
        bool sw = sp.n > sp.m;
        if (sw ? narrow_fits(sp.n, sp.k, sp.m) : narrow_fits(sp.m, sp.k, sp.n)) {
          ch.kind = 3;
          ch.cfg = 0;
          ch.swap = sw;
        }
      }
      r->choice[mode].push_back(ch);
    }
  r->needs_grad.assign(p->tensors.size(), 0);
  for (size_t v = 0; v < p->tensors.size(); ++v) {
    if ((int)v < p->L)
      r->needs_grad[v] = p->leaves[v].param >= 0;
    else {
      const StepPlan& sp = p->steps[v - p->L];
      r->needs_grad[v] = r->needs_grad[sp.left] || r->needs_grad[sp.right];
    }
  }
  // uploads (host vectors live in the plan / impl; synchronised below)
  HIPCHECK(hipMemcpyAsync(r->ws + r->lay.leafdata, p->leaf_data.data(), (size_t)p->leaf_elems * 8,
                          hipMemcpyHostToDevice, r->st));
  HIPCHECK(hipMemcpyAsync(r->ws + r->lay.gd_fwd, r->gd_fwd.data(), r->gd_fwd.size() * sizeof(GatherDesc),
                          hipMemcpyHostToDevice, r->st));
  if (grad) {
    HIPCHECK(hipMemcpyAsync(r->ws + r->lay.gd_grad, r->gd_grad.data(),
                            r->gd_grad.size() * sizeof(GatherDesc), hipMemcpyHostToDevice, r->st));
    HIPCHECK(hipMemcpyAsync(r->ws + r->lay.gd_gcot, r->gd_gcot.data(),
                            r->gd_gcot.size() * sizeof(GatherDesc), hipMemcpyHostToDevice, r->st));
  }
  if (r->n_pl)
    HIPCHECK(hipMemcpyAsync(r->ws + r->lay.pl, r->pl.data(), r->pl.size() * sizeof(ParamLeaf),
                            hipMemcpyHostToDevice, r->st));
  HIPCHECK(hipStreamSynchronize(r->st));
}

}  // namespace

extern "C" ltn_status ltn_bind(ltn_plan* p, void* d_ws, size_t bytes, int32_t grad, void* stream) {
  return guarded([&] {
    require(p != nullptr, "plan is NULL");
    require(d_ws != nullptr, "workspace is NULL");
    require(((uintptr_t)d_ws & 255) == 0, "workspace must be 256-byte aligned");
    // grid.y limit of the gather; no batch larger than the slice count
    const int B = fit_batch(p, bytes, grad, 4096);
    if (B == 0)
      fail(LTN_E_NOMEM, "workspace of " + std::to_string(bytes) + " bytes is below the " +
                            std::to_string(layout(p, 1, grad).total) + " needed for one slice");
    runtime_free(p);
    auto r = new ltn_plan_impl();
    p->rt = r;
    bind_state(p, r, reinterpret_cast<char*>(d_ws), bytes, grad, reinterpret_cast<hipStream_t>(stream), B);
  });
}

static void build_grad_seq(ltn_plan* p);

static ltn_status execute_impl(ltn_plan* p, const uint64_t* ids, uint64_t begin, uint64_t n,
                               bool range, int32_t mode, void* d_out) {
  return guarded([&] {
    auto& r = rt(p);
    check_mode(mode);
    require(d_out != nullptr, "d_out is NULL");
    const int ns = (int)p->sliced.size();
    if (range) {
      require(begin <= n, "range end before begin");
      require(ns >= 64 || n <= (1ull << ns), "slice range beyond 2^|S|");
      n = n - begin;
    } else {
      require(n == 0 || ids != nullptr, "slice_ids is NULL");
      if (ns < 64)
        for (uint64_t i = 0; i < n; ++i)
          require(ids[i] < (1ull << ns), "slice id " + std::to_string(ids[i]) + " is not below 2^|S|");
    }
    r.fwd_kept = false;
    if (r.grad && mode == LTN_C64 && n >= 1 && n <= (uint64_t)r.B) {
      // a plan bound for gradients runs a one-batch forward in its gradient
      // arena, whose tensors then stay for ltn_execute_grad on the same ids
      const int nb = (int)n;
      if (!r.gseq_valid) build_grad_seq(p);
      set_ids(p, range ? nullptr : ids, begin, nb, range);
      if (nb == r.B)
        launch_captured(p, r.ggraph[0], r.ggraph_src[0], [&] { enqueue_forward(p, nb, true, LTN_C64); });
      else
        enqueue_forward(p, nb, true, LTN_C64);
      enqueue_reduce(p, nb, true, reinterpret_cast<double*>(d_out));
      check_launch();
      r.fwd_ids.resize(n);
      for (uint64_t i = 0; i < n; ++i) r.fwd_ids[i] = range ? begin + i : ids[i];
      r.fwd_kept = true;
      return;
    }
    for (uint64_t off = 0; off < n; off += (uint64_t)r.B) {
      int nb = (int)std::min<uint64_t>((uint64_t)r.B, n - off);
      set_ids(p, range ? nullptr : ids + off, begin + off, nb, range);
      run_batch(p, nb, mode, reinterpret_cast<double*>(d_out));
    }
  });
}

extern "C" ltn_status ltn_execute(ltn_plan* p, const uint64_t* ids, uint64_t n, int32_t mode,
                                  void* d_out) {
  return execute_impl(p, ids, 0, n, false, mode, d_out);
}

extern "C" ltn_status ltn_execute_range(ltn_plan* p, uint64_t begin, uint64_t end, int32_t mode,
                                        void* d_out) {
  return execute_impl(p, nullptr, begin, end, true, mode, d_out);
}

// Device memory of the library's own, for callers that cannot allocate:
// one fixed array per GPU, held until the process ends. Host code never
// uses the array's name as an address (on the host it is only a handle);
// it uses the device address hipGetSymbolAddress returns for the current
// device, fetched once per device.
static __device__ __align__(256) char scratch[LTN_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

char* scratch_ptr() {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  require(dev >= 0 && dev < kMaxDevices, "device ordinal above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    require(ptr != nullptr, "no device address for the scratch array");
    g_scratch_ptr[dev] = reinterpret_cast<char*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" ltn_status ltn_execute_scratch(ltn_plan* p, const uint64_t* ids, uint64_t n, int32_t mode,
                                          void* d_out, void* stream) {
  return guarded([&] {
    require(p != nullptr, "plan is NULL");
    check_mode(mode);
    require(d_out != nullptr, "d_out is NULL");
    require(n == 0 || ids != nullptr, "slice_ids is NULL");
    const int ns = (int)p->sliced.size();
    if (ns < 64)
      for (uint64_t i = 0; i < n; ++i)
        require(ids[i] < (1ull << ns), "slice id " + std::to_string(ids[i]) + " is not below 2^|S|");
    if (n == 0) return;
    const int B = fit_batch(p, LTN_SCRATCH_BYTES, 0, (int)std::min<uint64_t>(n, 4096));
    if (B == 0)
      fail(LTN_E_NOMEM, "one slice needs " + std::to_string(layout(p, 1, 0).total) +
                            " bytes of workspace; the library's scratch holds " +
                            std::to_string((size_t)LTN_SCRATCH_BYTES));
    char* ws = scratch_ptr();
    // a state of this call only: the plan's own binding (if any) is kept
    ltn_plan_impl tmp;
    ltn_plan_impl* bound = p->rt;
    p->rt = &tmp;
    try {
      bind_state(p, &tmp, ws, LTN_SCRATCH_BYTES, 0, reinterpret_cast<hipStream_t>(stream), B);
      build_fwd_seq(p, mode);
      for (uint64_t off = 0; off < n; off += (uint64_t)B) {
        const int nb = (int)std::min<uint64_t>((uint64_t)B, n - off);
        set_ids(p, ids + off, 0, nb, false);
        enqueue_forward(p, nb, false, mode);
        enqueue_reduce(p, nb, false, reinterpret_cast<double*>(d_out));
        check_launch();
      }
    } catch (...) {
      p->rt = bound;
      throw;
    }
    p->rt = bound;
  });
}

extern "C" ltn_status ltn_set_params(ltn_plan* p, const double* d_angles) {
  return guarded([&] {
    auto& r = rt(p);
    require(r.n_pl == 0 || d_angles != nullptr, "d_angles is NULL");
    if (r.n_pl == 0) return;
    r.fwd_kept = false;
    double* ang = reinterpret_cast<double*>(r.ws + r.lay.angles);
    HIPCHECK(hipMemcpyAsync(ang, d_angles, (size_t)p->n_params * sizeof(double),
                            hipMemcpyDeviceToDevice, r.st));
    launch_u3_build(reinterpret_cast<const ParamLeaf*>(r.ws + r.lay.pl), r.n_pl, ang,
                    reinterpret_cast<float2*>(r.ws + r.lay.leafdata), r.st);
    check_launch();
  });
}

// One adjoint product in the forward form: C[merge(m, n)] = sum_k
// X[m 2^k + k] Y[n 2^k + k] over a batch of nb slices, on the complex64
// MFMA GEMM when a tile fits (either operand role), else the narrow kernel,
// else the generic kernel.
uint32_t adj_key(int m, int k, int n) { return (uint32_t)m | (uint32_t)k << 8 | (uint32_t)n << 16; }

static void nt_gemm(ltn_plan* p, const float2* X, int64_t sX, const float2* Y, int64_t sY, float2* C,
                    int64_t sC, int m, int k, int n, uint64_t cmask, int nb, int sw, int cfg) {
  const uint64_t full = (m + n) >= 64 ? ~0ull : ((1ull << (m + n)) - 1);
  GemmDesc d{};
  d.A = sw ? Y : X;
  d.B = sw ? X : Y;
  d.C = C;
  d.sA = sw ? sY : sX;
  d.sB = sw ? sX : sY;
  d.sC = sC;
  d.m = sw ? n : m;
  d.n = sw ? m : n;
  d.k = k;
  d.cmask = sw ? (~cmask & full) : cmask;
  d.nb = nb;
  d.cfg = cfg;
  launch_cgemm(d, LTN_C64, p->rt->st);
}

// The same product on a split-K tile (partials in the workspace's split-K
// buffer, which the layout sizes for the adjoint products of gradient plans).
static void nt_splitk(ltn_plan* p, const float2* X, int64_t sX, const float2* Y, int64_t sY, float2* C,
                      int64_t sC, int m, int k, int n, uint64_t cmask, int nb, int sw, int cfg) {
  auto& r = *p->rt;
  const uint64_t full = (m + n) >= 64 ? ~0ull : ((1ull << (m + n)) - 1);
  GemmDesc d{};
  d.A = sw ? Y : X;
  d.B = sw ? X : Y;
  d.C = C;
  d.sA = sw ? sY : sX;
  d.sB = sw ? sX : sY;
  d.sC = sC;
  d.m = sw ? n : m;
  d.n = sw ? m : n;
  d.k = k;
  d.cmask = sw ? (~cmask & full) : cmask;
  d.nb = nb;
  d.cfg = cfg;
  d.part = reinterpret_cast<float2*>(r.ws + r.lay.splitk);
  launch_cgemm_splitk(d, r.st);
}

static void enqueue_nt(ltn_plan* p, const float2* X, int64_t sX, const float2* Y, int64_t sY,
                       float2* C, int64_t sC, int m, int k, int n, uint64_t cmask, int nb) {
  auto& r = *p->rt;
  const uint64_t full = (m + n) >= 64 ? ~0ull : ((1ull << (m + n)) - 1);
  const auto tuned = r.adj.find(adj_key(m, k, n));
  if (tuned != r.adj.end() && tuned->second.kind == 1) {
    nt_gemm(p, X, sX, Y, sY, C, sC, m, k, n, cmask, nb, tuned->second.swap, tuned->second.cfg);
    return;
  }
  if (tuned != r.adj.end() && tuned->second.kind == 5) {
    nt_splitk(p, X, sX, Y, sY, C, sC, m, k, n, cmask, nb, tuned->second.swap, tuned->second.cfg);
    return;
  }
  for (int sw = 0; sw < 2; ++sw) {
    const int mm = sw ? n : m, nn = sw ? m : n;
    const int cfg = default_cfg(mm, k, nn, LTN_C64);
    if (cfg >= 0 && mm >= 5 && nn >= 5) {
      nt_gemm(p, X, sX, Y, sY, C, sC, m, k, n, cmask, nb, sw, cfg);
      return;
    }
  }
  if (m + n >= 12) {
    const bool sw = n > m;
    if (sw ? narrow_fits(n, k, m) : narrow_fits(m, k, n)) {
      NarrowDesc d{};
      d.A = sw ? Y : X;
      d.B = sw ? X : Y;
      d.C = C;
      d.sA = sw ? sY : sX;
      d.sB = sw ? sX : sY;
      d.sC = sC;
      d.m = sw ? n : m;
      d.n = sw ? m : n;
      d.k = k;
      d.cmask = sw ? (~cmask & full) : cmask;
      d.nb = nb;
      launch_narrow(d, r.st);
      return;
    }
  }
  GenericDesc g{};
  g.P = X;
  g.Q = Y;
  g.out = C;
  g.sP = sX;
  g.sQ = sY;
  g.sO = sC;
  g.xb = m;
  g.yb = n;
  g.zb = k;
  g.px = ((1ull << m) - 1) << k;
  g.pz = (1ull << k) - 1;
  g.qy = ((1ull << n) - 1) << k;
  g.qz = (1ull << k) - 1;
  g.ox = cmask;
  g.oy = ~cmask & full;
  g.nb = nb;
  launch_generic(g, default_tk(k, (1ull << (m + n)) * (uint64_t)nb), r.st);
}

static PermuteDesc plan_permute(int32_t rank, const int32_t* perm, int64_t batch, bool conj);

// Bit permutation of a batch of nb tensors (slice stride 2^rank), optionally
// conjugated, into `out`; returns the tensor to read (the input itself for
// the identity without conjugation).
static const float2* enqueue_perm(ltn_plan* p, const float2* in, float2* out,
                                  const std::vector<int32_t>& perm, int nb, bool conj) {
  bool ident = !conj;
  for (size_t j = 0; j < perm.size() && ident; ++j) ident = perm[j] == (int32_t)j;
  if (ident) return in;
  PermuteDesc d = plan_permute((int32_t)perm.size(), perm.data(), nb, conj);
  launch_permute(in, out, d, p->rt->st);
  return out;
}

// Adjoint of a small step for one operand (which 0: A, 1: B) on the
// generic kernel: the output cotangent times the other operand, conjugated,
// summed over the other operand's free bits; operands read in place.
static GenericDesc adj_generic_desc(ltn_plan* p, int s, int which, int nb, int* tk) {
  const StepPlan& sp = p->steps[s];
  const TensorPlan &ta = p->tensors[sp.a], &tb = p->tensors[sp.b], &tc = p->tensors[sp.out];
  const uint64_t cm = sp.c_mask_a, full = (1ull << (sp.m + sp.n)) - 1;
  GenericDesc g{};
  g.P = arena_ptr(p, tc.gcot);
  g.sP = int64_t(1) << tc.rank;
  g.yb = sp.k;
  g.qy = (1ull << sp.k) - 1;
  g.oy = (1ull << sp.k) - 1;
  g.conjQ = 1;
  g.nb = nb;
  if (which == 0) {
    g.Q = arena_ptr(p, tb.goff);
    g.out = arena_ptr(p, ta.gcot);
    g.sQ = int64_t(1) << tb.rank;
    g.sO = int64_t(1) << ta.rank;
    g.xb = sp.m;
    g.zb = sp.n;
    g.px = cm;
    g.pz = ~cm & full;
    g.qz = ((1ull << sp.n) - 1) << sp.k;
    g.ox = ((1ull << sp.m) - 1) << sp.k;
    *tk = default_tk(sp.n, (1ull << (sp.m + sp.k)) * (uint64_t)nb);
  } else {
    g.Q = arena_ptr(p, ta.goff);
    g.out = arena_ptr(p, tb.gcot);
    g.sQ = int64_t(1) << ta.rank;
    g.sO = int64_t(1) << tb.rank;
    g.xb = sp.n;
    g.zb = sp.m;
    g.px = ~cm & full;
    g.pz = cm;
    g.qz = ((1ull << sp.m) - 1) << sp.k;
    g.ox = ((1ull << sp.n) - 1) << sp.k;
    *tk = default_tk(sp.m, (1ull << (sp.n + sp.k)) * (uint64_t)nb);
  }
  return g;
}

// Adjoint of step s (operand cotangents from the output's cotangent).
static void enqueue_adjoint_step(ltn_plan* p, int s, int nb) {
  auto& r = *p->rt;
  const StepPlan& sp = p->steps[s];
  if (!r.needs_grad[sp.out]) return;
  const TensorPlan &ta = p->tensors[sp.a], &tb = p->tensors[sp.b], &tc = p->tensors[sp.out];
  const uint64_t cm = sp.c_mask_a;
  {
    // small steps: one generic kernel per operand, reading the operands
    // in place (strided) and conjugating the second one
    if (sp.m + sp.n + sp.k <= 16) {
      for (int which = 0; which < 2; ++which)
        if (r.needs_grad[which ? sp.b : sp.a]) {
          int tk = 1;
          GenericDesc g = adj_generic_desc(p, s, which, nb, &tk);
          launch_generic(g, tk, r.st);
        }
      return;
    }
    // adjoint products in the forward form: the output cotangent
    // and the other operand are permuted so that the summed bits are
    // lowest (and the operand conjugated), then one GEMM per operand
    float2* Xs = reinterpret_cast<float2*>(r.ws + r.lay.gscr_c);
    float2* Ys = reinterpret_cast<float2*>(r.ws + r.lay.gscr);
    const int rc = sp.m + sp.n;
    // positions of the m bits (in order) and the n bits of the output
    std::vector<int> mpos, npos;
    for (int j = 0; j < rc; ++j) ((cm >> j) & 1 ? mpos : npos).push_back(j);
    if (r.needs_grad[sp.a]) {
      // dA[m][k] = sum_n dC[merge(m, n)] conj(B[n][k])
      std::vector<int32_t> pc(rc), pb(sp.k + sp.n);
      for (int i = 0; i < sp.m; ++i) pc[mpos[i]] = sp.n + i;
      for (int i = 0; i < sp.n; ++i) pc[npos[i]] = i;
      for (int j = 0; j < sp.k; ++j) pb[j] = sp.n + j;
      for (int i = 0; i < sp.n; ++i) pb[sp.k + i] = i;
      const float2* X = enqueue_perm(p, arena_ptr(p, tc.gcot), Xs, pc, nb, false);
      enqueue_perm(p, arena_ptr(p, tb.goff), Ys, pb, nb, true);
      enqueue_nt(p, X, int64_t(1) << rc, Ys, int64_t(1) << tb.rank, arena_ptr(p, ta.gcot),
                 int64_t(1) << ta.rank, sp.m, sp.n, sp.k, ((1ull << sp.m) - 1) << sp.k, nb);
    }
    if (r.needs_grad[sp.b]) {
      // dB[n][k] = sum_m dC[merge(m, n)] conj(A[m][k])
      std::vector<int32_t> pc(rc), pa(sp.k + sp.m);
      for (int i = 0; i < sp.m; ++i) pc[mpos[i]] = i;
      for (int i = 0; i < sp.n; ++i) pc[npos[i]] = sp.m + i;
      for (int j = 0; j < sp.k; ++j) pa[j] = sp.m + j;
      for (int i = 0; i < sp.m; ++i) pa[sp.k + i] = i;
      const float2* X = enqueue_perm(p, arena_ptr(p, tc.gcot), Xs, pc, nb, false);
      enqueue_perm(p, arena_ptr(p, ta.goff), Ys, pa, nb, true);
      enqueue_nt(p, X, int64_t(1) << rc, Ys, int64_t(1) << ta.rank, arena_ptr(p, tb.gcot),
                 int64_t(1) << tb.rank, sp.n, sp.m, sp.k, ((1ull << sp.n) - 1) << sp.k, nb);
    }
  }
}

// Adjoint sweep of one batch (steps in reverse order), then the leaf
// cotangents accumulated into the per-leaf FP64 sums. Every pointer is in
// the bound workspace, so a full batch can run from a captured graph.
static void enqueue_backward(ltn_plan* p, int nb) {
  auto& r = *p->rt;
  double* lg = reinterpret_cast<double*>(r.ws + r.lay.leafgrad);
  const GatherDesc* gcot = reinterpret_cast<const GatherDesc*>(r.ws + r.lay.gd_gcot);
  const uint64_t* dids = reinterpret_cast<const uint64_t*>(r.ws + r.lay.ids);
  if (r.gseq_valid) {
    const GenericDesc* dd = reinterpret_cast<const GenericDesc*>(r.ws + r.lay.gdesc);
    for (const auto& it : r.gseq_bwd) {
      if (it.what == 1)
        launch_generic_multi(dd + it.off, it.count, it.max_outs, nb, it.tk, r.st);
      else
        enqueue_adjoint_step(p, it.step, nb);
    }
  } else {
    for (int s = (int)p->steps.size() - 1; s >= 0; --s) enqueue_adjoint_step(p, s, nb);
  }
  launch_leaf_cot_accumulate(reinterpret_cast<const ParamLeaf*>(r.ws + r.lay.pl), r.n_pl, gcot,
                             arena_ptr(p, 0), dids, nb, lg, r.st);
}

// Gradient launch sequence. The gradient arena gives every tensor and every
// cotangent a place of its own, so consecutive generic contractions can
// share one launch as long as none of them reads what another one writes:
// forward, a step that consumes a tensor the run produces starts a new run;
// backward (reverse order), a step whose output cotangent the run writes
// does. Other kernels keep their place between the runs. The descriptors
// (for the bound batch size; the launch passes the actual one) are copied
// to the workspace here, outside any capture.
static void build_grad_seq(ltn_plan* p) {
  auto& r = *p->rt;
  using Item = ltn_plan_impl::GradItem;
  r.gseq_descs.clear();
  r.gseq_fwd.clear();
  r.gseq_bwd.clear();
  std::vector<std::pair<GenericDesc, int>> run;
  std::vector<char> written(p->tensors.size(), 0);
  std::vector<int> wlist;
  auto flush = [&](std::vector<Item>& seq) {
    for (int tk : {1, 8, 64}) {
      Item it;
      it.what = 1;
      it.tk = tk;
      it.off = (int)r.gseq_descs.size();
      for (auto& e : run)
        if (e.second == tk) {
          r.gseq_descs.push_back(e.first);
          it.max_outs = std::max<uint64_t>(it.max_outs, 1ull << (e.first.xb + e.first.yb));
        }
      it.count = (int)r.gseq_descs.size() - it.off;
      if (it.count) seq.push_back(it);
    }
    run.clear();
    for (int t : wlist) written[t] = 0;
    wlist.clear();
  };
  auto single = [&](std::vector<Item>& seq, int what, int s) {
    flush(seq);
    Item it;
    it.what = what;
    it.step = s;
    seq.push_back(it);
  };
  for (int s = 0; s < (int)p->steps.size(); ++s) {
    const StepPlan& sp = p->steps[s];
    const auto& ch = r.choice[LTN_C64][s];
    if (ch.kind != 0) {
      single(r.gseq_fwd, 0, s);
      continue;
    }
    if (written[sp.a] || written[sp.b]) flush(r.gseq_fwd);
    run.push_back({step_generic_desc(p, s, r.B, true, LTN_C64), ch.tk});
    written[sp.out] = 1;
    wlist.push_back(sp.out);
  }
  flush(r.gseq_fwd);
  for (int s = (int)p->steps.size() - 1; s >= 0; --s) {
    const StepPlan& sp = p->steps[s];
    if (!r.needs_grad[sp.out]) continue;
    if (sp.m + sp.n + sp.k > 16) {
      single(r.gseq_bwd, 2, s);
      continue;
    }
    if (written[sp.out]) flush(r.gseq_bwd);
    for (int which = 0; which < 2; ++which) {
      const int t = which ? sp.b : sp.a;
      if (!r.needs_grad[t]) continue;
      int tk = 1;
      run.push_back({adj_generic_desc(p, s, which, r.B, &tk), tk});
      written[t] = 1;
      wlist.push_back(t);
    }
  }
  flush(r.gseq_bwd);
  require(r.gseq_descs.size() <= 3 * p->steps.size(), "gradient descriptor area too small");
  if (!r.gseq_descs.empty())
    HIPCHECK(hipMemcpyAsync(r.ws + r.lay.gdesc, r.gseq_descs.data(), r.gseq_descs.size() * sizeof(GenericDesc),
                            hipMemcpyHostToDevice, r.st));
  // the host array may be rebuilt by a later call: let the copy finish
  HIPCHECK(hipStreamSynchronize(r.st));
  r.gseq_valid = true;
}

extern "C" ltn_status ltn_execute_grad(ltn_plan* p, const uint64_t* ids, uint64_t n, int32_t mode,
                                       const void* d_cot, void* d_out, double* d_angle_grad) {
  return guarded([&] {
    auto& r = rt(p);
    check_mode(mode);
    if (mode != LTN_C64) fail(LTN_E_UNSUPPORTED, "gradients run in complex64 only");
    require(r.grad, "plan was bound without gradient workspace");
    require(d_cot && d_angle_grad, "NULL argument");
    require(n == 0 || ids, "slice_ids is NULL");
    const int ns = (int)p->sliced.size();
    if (ns < 64)
      for (uint64_t i = 0; i < n; ++i) require(ids[i] < (1ull << ns), "slice id is not below 2^|S|");
    double* lg = reinterpret_cast<double*>(r.ws + r.lay.leafgrad);
    if (!r.gseq_valid) build_grad_seq(p);
    // the forward of these very slices (same parameters) is still in the
    // gradient arena after a one-batch ltn_execute: it is not recomputed
    const bool kept = r.fwd_kept && n == r.fwd_ids.size() && std::equal(ids, ids + n, r.fwd_ids.begin());
    r.fwd_kept = false;
    launch_fill_zero(lg, al((size_t)r.n_pl * 64), r.st);
    const uint64_t* dids = reinterpret_cast<const uint64_t*>(r.ws + r.lay.ids);
    // full batches run the recomputed forward and the adjoint sweep from two
    // captured graphs; the cotangent and output pointers stay outside them
    for (uint64_t off = 0; off < n; off += (uint64_t)r.B) {
      int nb = (int)std::min<uint64_t>((uint64_t)r.B, n - off);
      if (!kept) {
        set_ids(p, ids + off, 0, nb, false);
        if (nb == r.B)
          launch_captured(p, r.ggraph[0], r.ggraph_src[0], [&] { enqueue_forward(p, nb, true, LTN_C64); });
        else
          enqueue_forward(p, nb, true, LTN_C64);
      }
      if (d_out) enqueue_reduce(p, nb, true, reinterpret_cast<double*>(d_out));
      const TensorPlan& root = p->tensors[p->root];
      launch_root_cotangent(reinterpret_cast<const double*>(d_cot), root.rank, p->out_mask,
                            r.sl_bits.data(), r.out_bits.data(), (int)r.sl_bits.size(), dids, nb,
                            arena_ptr(p, root.gcot), r.st);
      if (nb == r.B)
        launch_captured(p, r.ggraph[1], r.ggraph_src[1], [&] { enqueue_backward(p, nb); });
      else
        enqueue_backward(p, nb);
      check_launch();
    }
    launch_u3_adjoint(reinterpret_cast<const ParamLeaf*>(r.ws + r.lay.pl), r.n_pl,
                      reinterpret_cast<const double*>(r.ws + r.lay.angles), lg, d_angle_grad, r.st);
    check_launch();
  });
}

namespace {

std::string tune_key(int mode, const StepPlan& sp, int B) {
  std::ostringstream o;
  o << "m" << mode << "_" << sp.m << "_" << sp.k << "_" << sp.n << "_" << (sp.c_mask_a & 1) << "_b" << B;
  return o.str();
}

std::map<std::string, std::pair<int, int>> read_cache(const char* path) {
  std::map<std::string, std::pair<int, int>> c;
  if (!path) return c;
  std::ifstream f(path);
  if (!f) return c;
  std::stringstream ss;
  ss << f.rdbuf();
  std::string s = ss.str();
  // entries look like "key": [a, b]
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    size_t e = s.find('"', pos + 1);
    if (e == std::string::npos) break;
    std::string key = s.substr(pos + 1, e - pos - 1);
    size_t lb = s.find('[', e), rb = s.find(']', e);
    if (lb == std::string::npos || rb == std::string::npos) break;
    int a = 0, b = 0;
    if (sscanf(s.c_str() + lb + 1, "%d , %d", &a, &b) == 2) c[key] = {a, b};
    pos = rb + 1;
  }
  return c;
}

void write_cache(const char* path, const std::map<std::string, std::pair<int, int>>& c) {
  if (!path) return;
  std::ofstream f(path);
  f << "{\n";
  size_t i = 0;
  for (auto& kv : c)
    f << "  \"" << kv.first << "\": [" << kv.second.first << ", " << kv.second.second << "]"
      << (++i < c.size() ? ",\n" : "\n");
  f << "}\n";
}

float time_step(ltn_plan* p, int s, int reps, int mode, bool warm = true) {
  auto& r = *p->rt;
  hipEvent_t a, b;
  HIPCHECK(hipEventCreate(&a));
  HIPCHECK(hipEventCreate(&b));
  if (warm) enqueue_step(p, s, r.B, false, mode);  // untimed warm-up launch
  HIPCHECK(hipEventRecord(a, r.st));
  for (int i = 0; i < reps; ++i) enqueue_step(p, s, r.B, false, mode);
  HIPCHECK(hipEventRecord(b, r.st));
  HIPCHECK(hipEventSynchronize(b));
  float ms = 0;
  HIPCHECK(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  check_launch();
  return ms / reps;
}

void drop_graphs(ltn_plan* p) {
  auto& r = *p->rt;
  for (int m = 0; m < 3; ++m) {
    if (r.graph[m]) (void)hipGraphExecDestroy(r.graph[m]);
    if (r.graph_src[m]) (void)hipGraphDestroy(r.graph_src[m]);
    r.graph[m] = nullptr;
    r.graph_src[m] = nullptr;
  }
  for (int m = 0; m < 2; ++m) {
    if (r.ggraph[m]) (void)hipGraphExecDestroy(r.ggraph[m]);
    if (r.ggraph_src[m]) (void)hipGraphDestroy(r.ggraph_src[m]);
    r.ggraph[m] = nullptr;
    r.ggraph_src[m] = nullptr;
  }
  r.gseq_valid = false;  // kernel choices or fusion may have changed
  r.fwd_kept = false;
  for (int m = 0; m < 3; ++m) r.fseq_valid[m] = false;
}

// Average duration of `launch` over reps launches (after one untimed launch
// when warm), with HIP events on the plan's stream.
template <typename F>
float time_launch(ltn_plan* p, F&& launch, int reps, bool warm) {
  auto& r = *p->rt;
  hipEvent_t a, b;
  HIPCHECK(hipEventCreate(&a));
  HIPCHECK(hipEventCreate(&b));
  if (warm) launch();
  HIPCHECK(hipEventRecord(a, r.st));
  for (int i = 0; i < reps; ++i) launch();
  HIPCHECK(hipEventRecord(b, r.st));
  HIPCHECK(hipEventSynchronize(b));
  float ms = 0;
  HIPCHECK(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  check_launch();
  return ms / reps;
}

// Tile choice for the adjoint products of the gradient sweep (plans bound
// for gradients, complex64): every complex64 tile that fits each product
// shape in either operand role, against the fixed rule, timed like the
// forward steps on the gradient scratch buffers (the values do not matter:
// every product overwrites its output). Cache entries "g0_m_k_n_bB":
// [1000 + cfg, swap], or [-1, 0] for the fixed rule.
void tune_adjoint(ltn_plan* p, std::map<std::string, std::pair<int, int>>& cache, bool& dirty) {
  auto& r = *p->rt;
  using Choice = ltn_plan_impl::Choice;
  float2* Xs = reinterpret_cast<float2*>(r.ws + r.lay.gscr_c);
  float2* Ys = reinterpret_cast<float2*>(r.ws + r.lay.gscr);
  for (const StepPlan& sp : p->steps) {
    if (!r.needs_grad[sp.out] || sp.m + sp.n + sp.k <= 16) continue;
    const TensorPlan &ta = p->tensors[sp.a], &tb = p->tensors[sp.b];
    const int rc = sp.m + sp.n;
    for (int which = 0; which < 2; ++which) {
      if (!r.needs_grad[which ? sp.b : sp.a]) continue;
      // dA: (m, n, k) with B's layout; dB: (n, m, k) with A's layout
      const int m = which ? sp.n : sp.m, k = which ? sp.m : sp.n, n = sp.k;
      const TensorPlan& other = which ? ta : tb;
      const TensorPlan& self = which ? tb : ta;
      float2* C = arena_ptr(p, self.gcot);
      const uint64_t cmask = ((1ull << m) - 1) << n;
      const uint32_t key = adj_key(m, k, n);
      if (r.adj.count(key)) continue;
      std::ostringstream o;
      o << "g0_" << m << "_" << k << "_" << n << "_b" << r.B;
      const auto it = cache.find(o.str());
      Choice pick;  // kind 0: the fixed rule
      if (it != cache.end()) {
        const int kind = it->second.first >= 1000 ? it->second.first / 1000 : 0;
        const int cfg = it->second.first % 1000, sw = it->second.second;
        if (kind == 1 && (sw ? gemm_config_fits(cfg, n, k, m, LTN_C64) : gemm_config_fits(cfg, m, k, n, LTN_C64))) {
          pick.kind = 1;
          pick.cfg = cfg;
          pick.swap = sw;
        } else if (kind == 5 && (sw ? splitk_config_fits(cfg, n, k, m) : splitk_config_fits(cfg, m, k, n))) {
          pick.kind = 5;
          pick.cfg = cfg;
          pick.swap = sw;
        }
      } else {
        auto run = [&](const Choice& c) {
          if (c.kind == 1)
            nt_gemm(p, Xs, int64_t(1) << rc, Ys, int64_t(1) << other.rank, C, int64_t(1) << self.rank,
                    m, k, n, cmask, r.B, c.swap, c.cfg);
          else if (c.kind == 5)
            nt_splitk(p, Xs, int64_t(1) << rc, Ys, int64_t(1) << other.rank, C, int64_t(1) << self.rank,
                      m, k, n, cmask, r.B, c.swap, c.cfg);
          else {
            r.adj.erase(key);
            enqueue_nt(p, Xs, int64_t(1) << rc, Ys, int64_t(1) << other.rank, C, int64_t(1) << self.rank,
                       m, k, n, cmask, r.B);
          }
        };
        std::vector<Choice> cands(1);
        for (int sw = 0; sw < 2; ++sw)
          for (int c = 0; c < gemm_config_count(LTN_C64); ++c)
            if (sw ? gemm_config_fits(c, n, k, m, LTN_C64) : gemm_config_fits(c, m, k, n, LTN_C64)) {
              Choice ch;
              ch.kind = 1;
              ch.cfg = c;
              ch.swap = sw;
              cands.push_back(ch);
            }
        for (int sw = 0; sw < 2; ++sw)
          for (int c = 0; c < splitk_config_count(); ++c)
            if (sw ? splitk_config_fits(c, n, k, m) : splitk_config_fits(c, m, k, n)) {
              Choice ch;
              ch.kind = 5;
              ch.cfg = c;
              ch.swap = sw;
              cands.push_back(ch);
            }
        float best = 1e30f;
        bool first = true;
        for (auto& c : cands) {
          float ms = time_launch(p, [&] { run(c); }, 1, first);
          first = false;
          if (ms > 2.0f * best) continue;
          if (ms < 2.0f)
            ms = std::min(ms, time_launch(p, [&] { run(c); }, 3, false));
          else if (ms < 1.05f * best)
            ms = std::min(ms, time_launch(p, [&] { run(c); }, 1, false));
          if (ms < best) {
            best = ms;
            pick = c;
          }
        }
        cache[o.str()] = pick.kind > 0 ? std::make_pair(1000 * pick.kind + pick.cfg, pick.swap) : std::make_pair(-1, 0);
        dirty = true;
      }
      r.adj[key] = pick;
    }
  }
}

}  // namespace

// Candidates: every MFMA tile configuration that fits the step in either
// operand role (split tiles first in the split modes, then complex64 tiles),
// the narrow-step kernel in either role (k + n <= 10), the split-sum kernel
// (m, n <= 3), and the generic kernel with 1, 8 or 64 threads per output on
// small steps.
// Cache entries: [kind * 1000 + cfg, swap] for MFMA kinds, [-tk, 0] for the
// generic kernel.
extern "C" ltn_status ltn_autotune(ltn_plan* p, int32_t mode, const char* cache_path) {
  return guarded([&] {
    auto& r = rt(p);
    check_mode(mode);
    auto cache = read_cache(cache_path);
    bool dirty = false;
    using Choice = ltn_plan_impl::Choice;
    auto encode = [](const Choice& c) {
      return c.kind > 0 ? std::make_pair(c.kind * 1000 + c.cfg, c.swap) : std::make_pair(-c.tk, 0);
    };
    auto decode = [](std::pair<int, int> e) {
      Choice c;
      if (e.first >= 0) {
        c.kind = e.first / 1000;
        c.cfg = e.first % 1000;
        c.swap = e.second;
      } else {
        c.kind = 0;
        c.tk = -e.first;
      }
      return c;
    };
    // the synchronising time_step below must not run inside a capture
    // and a stale graph would keep the old kernels
    drop_graphs(p);
    // time on realistic values (power and clocks depend on the data): one
    // forward pass over slices 0.. fills every tensor of the arena, and in
    // split-fp16 mode the per-slice maxima (not needed when every step's
    // choice comes from the cache)
    bool all_cached = true;
    for (auto& sp : p->steps) all_cached = all_cached && cache.count(tune_key(mode, sp, r.B)) > 0;
    if (!all_cached) {
      set_ids(p, nullptr, 0, r.B, true);
      enqueue_forward(p, r.B, false, mode == LTN_C64 ? LTN_C64 : mode);
    }
    for (int s = 0; s < (int)p->steps.size(); ++s) {
      const StepPlan& sp = p->steps[s];
      std::string key = tune_key(mode, sp, r.B);
      auto it = cache.find(key);
      std::vector<Choice> cands;
      if (it != cache.end()) {
        cands.push_back(decode(it->second));
      } else {
        for (int kind : {2, 1}) {
          if (kind == 2 && mode == LTN_C64) continue;
          int km = kind == 2 ? mode : LTN_C64;
          for (int sw = 0; sw < 2; ++sw)
            for (int c = 0; c < gemm_config_count(km); ++c)
              if (sw ? gemm_config_fits(c, sp.n, sp.k, sp.m, km) : gemm_config_fits(c, sp.m, sp.k, sp.n, km)) {
                Choice ch;
                ch.kind = kind;
                ch.cfg = c;
                ch.swap = sw;
                cands.push_back(ch);
              }
        }
        for (int sw = 0; sw < 2; ++sw) {
          if (sw ? narrow_fits(sp.n, sp.k, sp.m) : narrow_fits(sp.m, sp.k, sp.n)) {
            Choice ch;
            ch.kind = 3;
            ch.cfg = 0;
            ch.swap = sw;
            cands.push_back(ch);
          }
          if (sw ? narrow_rows_fits(sp.n, sp.k, sp.m) : narrow_rows_fits(sp.m, sp.k, sp.n)) {
            Choice ch;
            ch.kind = 3;
            ch.cfg = 1;
            ch.swap = sw;
            cands.push_back(ch);
          }
        }
        if (skinny_fits(sp.m, sp.k, sp.n)) {
          Choice ch;
          ch.kind = 4;
          ch.cfg = 0;
          cands.push_back(ch);
        }
        for (int sw = 0; sw < 2; ++sw)
          for (int c = 0; c < splitk_config_count(); ++c)
            if (sw ? splitk_config_fits(c, sp.n, sp.k, sp.m) : splitk_config_fits(c, sp.m, sp.k, sp.n)) {
              Choice ch;
              ch.kind = 5;
              ch.cfg = c;
              ch.swap = sw;
              cands.push_back(ch);
            }
        // the generic kernel only competes on small steps (or when no tile fits)
        if (cands.empty() || (cands.size() == 1 && cands[0].kind == 4) || sp.m + sp.k + sp.n <= 22)
          for (int tk : {1, 8, 64})
            if (tk == 1 || (1 << sp.k) >= tk) {
              Choice ch;
              ch.tk = tk;
              cands.push_back(ch);
            }
      }
      // one launch of each candidate; clearly slower ones get no repeats,
      // short launches (timer and launch noise) three more, long ones one
      // more only when they come within 5 % of the best so far
      float best = 1e30f;
      Choice pick = cands[0];
      bool first = true;
      for (auto& c : cands) {
        r.choice[mode][s] = c;
        if (cands.size() == 1) break;
        float ms = time_step(p, s, 1, mode, first);
        first = false;
        if (ms > 2.0f * best) continue;
        if (ms < 2.0f)
          ms = std::min(ms, time_step(p, s, 3, mode, false));
        else if (ms < 1.05f * best)
          ms = std::min(ms, time_step(p, s, 1, mode, false));
        if (ms < best) {
          best = ms;
          pick = c;
        }
      }
      r.choice[mode][s] = pick;
      if (it == cache.end()) {
        cache[key] = encode(pick);
        dirty = true;
      }
    }
    if (mode == LTN_C64 && r.grad) tune_adjoint(p, cache, dirty);
    if (dirty) write_cache(cache_path, cache);
    HIPCHECK(hipStreamSynchronize(r.st));
  });
}

extern "C" ltn_status ltn_profile_steps(ltn_plan* p, uint64_t first, int32_t mode, float* ms_out) {
  return guarded([&] {
    auto& r = rt(p);
    check_mode(mode);
    require(ms_out != nullptr, "ms_out is NULL");
    r.fwd_kept = false;
    set_ids(p, nullptr, first, r.B, true);
    const GatherDesc* gd = reinterpret_cast<const GatherDesc*>(r.ws + r.lay.gd_fwd);
    uint32_t* scales = nullptr;
    if (mode == LTN_SPLIT_F16) {
      scales = reinterpret_cast<uint32_t*>(r.ws + r.lay.scales);
      launch_fill_zero(scales, al((size_t)r.B * p->tensors.size() * 4), r.st);
    }
    launch_gather(gd, (int)p->leaves.size(), r.gather_chunks, r.max_leaf_elems,
                  reinterpret_cast<const float2*>(r.ws + r.lay.leafdata), arena_ptr(p, 0),
                  reinterpret_cast<const uint64_t*>(r.ws + r.lay.ids), r.B, scales, r.B, r.st);
    std::vector<hipEvent_t> ev(p->steps.size() + 1);
    for (auto& e : ev) HIPCHECK(hipEventCreate(&e));
    HIPCHECK(hipEventRecord(ev[0], r.st));
    for (int s = 0; s < (int)p->steps.size(); ++s) {
      enqueue_step(p, s, r.B, false, mode);
      HIPCHECK(hipEventRecord(ev[s + 1], r.st));
    }
    HIPCHECK(hipEventSynchronize(ev.back()));
    for (int s = 0; s < (int)p->steps.size(); ++s) HIPCHECK(hipEventElapsedTime(&ms_out[s], ev[s], ev[s + 1]));
    for (auto& e : ev) (void)hipEventDestroy(e);
    check_launch();
  });
}

extern "C" ltn_status ltn_set_fusion(ltn_plan* p, int32_t enable) {
  return guarded([&] {
    require(p && p->rt, "plan is not bound", LTN_E_STATE);
    drop_graphs(p);
    p->rt->fuse = enable != 0;
  });
}

extern "C" ltn_status ltn_set_step_kernel(ltn_plan* p, int32_t step, int32_t mode, int32_t kind,
                                          int32_t cfg, int32_t swap, int32_t tk) {
  return guarded([&] {
    require(p && p->rt, "plan is not bound");
    require(step >= 0 && step < (int32_t)p->steps.size(), "step out of range");
    check_mode(mode);
    const StepPlan& sp = p->steps[step];
    const int m = swap ? sp.n : sp.m, n = swap ? sp.m : sp.n;
    ltn_plan_impl::Choice c;
    if (kind == 0) {
      require(tk == 1 || tk == 8 || tk == 64, "tk must be 1, 8 or 64");
      c.tk = tk;
    } else if (kind == 1 || kind == 2) {
      require(kind == 1 || mode != LTN_C64, "split GEMM kernels need a split mode");
      const int km = kind == 2 ? mode : LTN_C64;
      require(cfg >= 0 && cfg < gemm_config_count(km) && gemm_config_fits(cfg, m, sp.k, n, km),
              "tile configuration does not fit the step");
      c.kind = kind;
      c.cfg = cfg;
      c.swap = swap ? 1 : 0;
    } else if (kind == 3) {
      require(cfg == 0 || cfg == 1, "narrow kernel configuration must be 0 or 1");
      require(cfg == 0 ? narrow_fits(m, sp.k, n) : narrow_rows_fits(m, sp.k, n),
              "the narrow kernel does not fit the step");
      c.kind = 3;
      c.cfg = cfg;
      c.swap = swap ? 1 : 0;
    } else if (kind == 4) {
      require(skinny_fits(sp.m, sp.k, sp.n), "the split-sum kernel needs m <= 3 and n <= 3");
      c.kind = 4;
      c.cfg = 0;
    } else if (kind == 5) {
      require(splitk_config_fits(cfg, m, sp.k, n), "split-K tile configuration does not fit the step");
      c.kind = 5;
      c.cfg = cfg;
      c.swap = swap ? 1 : 0;
    } else {
      require(false, "unknown kernel kind");
    }
    drop_graphs(p);
    p->rt->choice[mode][step] = c;
  });
}

extern "C" ltn_status ltn_step_kernel(const ltn_plan* p, int32_t step, int32_t mode, int32_t* kind,
                                      int32_t* cfg, int32_t* swap, int32_t* tk) {
  return guarded([&] {
    require(p && p->rt, "plan is not bound");
    require(step >= 0 && step < (int32_t)p->steps.size(), "step out of range");
    check_mode(mode);
    const auto& c = p->rt->choice[mode][step];
    if (kind) *kind = c.kind;
    if (cfg) *cfg = c.kind > 0 ? c.cfg : -1;
    if (swap) *swap = c.swap;
    if (tk) *tk = c.tk;
  });
}

extern "C" const char* ltn_kernel_name(int32_t kind, int32_t cfg, int32_t mode) {
  if (mode < LTN_C64 || mode > LTN_SPLIT_BF16) return "?";
  switch (kind) {
    case 0: return "generic";
    case 1: return gemm_config_name(cfg, LTN_C64);
    case 2: return mode == LTN_C64 ? "?" : gemm_config_name(cfg, mode);
    case 3: return cfg == 0 ? "narrow_tile" : (cfg == 1 ? "narrow_rows" : "?");
    case 4: return cfg == 0 ? "split_sum" : "?";
    case 5: return splitk_config_name(cfg);
  }
  return "?";
}

// Tile plan of a bit permutation (see k_permute): the tile holds the lowest
// 5 source bits, the sources of the lowest 5 destination bits and then the
// next source bits up to 12; the LDS swizzle spreads one half-wave's reads
// in destination order over distinct banks.
static PermuteDesc plan_permute(int32_t rank, const int32_t* perm, int64_t batch, bool conj) {
  std::vector<int> inv(rank, -1);
  for (int j = 0; j < rank; ++j) {
    require(perm[j] >= 0 && perm[j] < rank && inv[perm[j]] < 0, "perm is not a permutation");
    inv[perm[j]] = j;
  }
  PermuteDesc d{};
  d.rank = rank;
  d.batch = batch;
  const int t = std::min(rank, 5);
  std::vector<char> in_tile(rank, 0);
  for (int j = 0; j < t; ++j) in_tile[j] = 1;          // lowest source bits
  for (int y = 0; y < t; ++y) in_tile[inv[y]] = 1;     // sources of the lowest destination bits
  int nt = 0;
  for (int j = 0; j < rank; ++j) nt += in_tile[j];
  for (int j = 0; j < rank && nt < std::min(rank, 12); ++j)
    if (!in_tile[j]) {
      in_tile[j] = 1;  // fill the tile up to 4096 elements with the next source bits
      ++nt;
    }
  std::vector<int> tsrc, outer;
  for (int j = 0; j < rank; ++j) (in_tile[j] ? tsrc : outer).push_back(j);
  d.n_tile = (int)tsrc.size();
  d.n_outer = (int)outer.size();
  for (int k = 0; k < d.n_tile; ++k) d.tile_src[k] = (int8_t)tsrc[k];
  // destination order of the tile bits
  std::vector<std::pair<int, int>> dt;
  for (int k = 0; k < d.n_tile; ++k) dt.push_back({perm[tsrc[k]], k});
  std::sort(dt.begin(), dt.end());
  for (int r = 0; r < d.n_tile; ++r) {
    d.tile_dst[r] = (int8_t)dt[r].first;
    d.dst_tile[r] = (int8_t)dt[r].second;
  }
  for (int k = 0; k < d.n_outer; ++k) {
    d.outer_src[k] = (int8_t)outer[k];
    d.outer_dst[k] = (int8_t)perm[outer[k]];
  }
  // LDS swizzle: the tile bits read by one half-wave in destination order
  // are dst_tile[0..4]; those at tile bit >= 5 each get a distinct low bit
  // not already among them, so the 32 slots differ in their low 5 bits.
  {
    const int nr = std::min(d.n_tile, 5);
    bool used[5] = {false, false, false, false, false};
    for (int r = 0; r < nr; ++r)
      if (d.dst_tile[r] < 5) used[d.dst_tile[r]] = true;
    int next = 0;
    for (int r = 0; r < nr; ++r)
      if (d.dst_tile[r] >= 5) {
        while (used[next]) ++next;
        used[next] = true;
        d.swz[d.dst_tile[r] - 5] = (uint8_t)(1u << next);
      }
  }
  d.flip = conj ? (1ull << 63) : 0;
  return d;
}

extern "C" ltn_status ltn_permute(const void* d_in, void* d_out, int32_t rank, const int32_t* perm,
                                  int64_t batch, void* stream) {
  return guarded([&] {
    require(d_in && d_out, "NULL buffer");
    require(d_in != d_out, "ltn_permute does not work in place");
    require(rank >= 0 && rank <= 40, "rank must be in 0..40");
    require(batch >= 1, "batch must be >= 1");
    require(rank == 0 || perm != nullptr, "perm is NULL");
    require(rank == 0 || ((uintptr_t)d_in % 16 == 0 && (uintptr_t)d_out % 16 == 0),
            "d_in and d_out must be 16-byte aligned");
    for (int j = 0; j < rank; ++j) require(perm[j] >= 0 && perm[j] < rank, "perm is not a permutation");
    std::vector<char> seen(rank, 0);
    for (int j = 0; j < rank; ++j) {
      require(!seen[perm[j]], "perm is not a permutation");
      seen[perm[j]] = 1;
    }
    PermuteDesc d = plan_permute(rank, perm, batch, false);
    launch_permute(reinterpret_cast<const float2*>(d_in), reinterpret_cast<float2*>(d_out), d,
                   reinterpret_cast<hipStream_t>(stream));
    check_launch();
  });
}
