// Host planner: greedy contraction path, contraction tree and its costs
// (Eq. (1), (2), (4)), the stem, lifetimes, the slice finder (Algorithm 1)
// with a fix-up for off-stem tensors, the slice refiner (Algorithms 2-4)
// and a greedy least-overhead slicer for comparison.
//
// Compiled with -ffp-contract=off: the greedy key is specified as a fixed
// sequence of IEEE double operations so that any implementation of the same
// rule makes the same choices.
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <unordered_map>

#include "common.h"

namespace ltn {

static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  uint64_t z = x;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double keyed_uniform(uint64_t seed, uint64_t step, uint64_t a, uint64_t b) {
  uint64_t h = splitmix64(seed);
  h = splitmix64(h ^ step);
  h = splitmix64(h ^ a);
  h = splitmix64(h ^ b);
  return (double)(h >> 11) * 0x1.0p-53;
}

static double pair_key(int rc, int ra, int rb, double alpha, double tau, double u) {
  double t1 = std::ldexp(1.0, ra) + std::ldexp(1.0, rb);
  double t2 = alpha * t1;
  double base = std::ldexp(1.0, rc) - t2;
  if (tau > 0.0) {
    double f = tau * u;
    if (base > 0.0)
      base = base * (1.0 + f);
    else
      base = base * (1.0 - f);
  }
  return base;
}

std::vector<int32_t> greedy(const std::vector<IdSet>& leaves, const IdSet& exclude, double alpha,
                            double tau, uint64_t seed) {
  const int32_t L = (int32_t)leaves.size();
  std::map<int32_t, IdSet> live;
  std::unordered_map<int32_t, std::vector<int32_t>> owner;
  for (int32_t i = 0; i < L; ++i) {
    live[i] = set_minus(leaves[i], exclude);
    for (int32_t x : live[i]) owner[x].push_back(i);
  }
  std::vector<int32_t> path;
  int32_t nxt = L;
  uint64_t step = 0;
  while (live.size() > 1) {
    bool have = false;
    double bk = 0;
    int32_t ba = 0, bb = 0;
    for (auto& kv : owner) {
      if (kv.second.size() != 2) continue;
      int32_t a = std::min(kv.second[0], kv.second[1]), b = std::max(kv.second[0], kv.second[1]);
      const IdSet& ia = live[a];
      const IdSet& ib = live[b];
      int shared = (int)set_and(ia, ib).size();
      int rc = (int)ia.size() + (int)ib.size() - 2 * shared;
      double u = tau > 0.0 ? keyed_uniform(seed, step, (uint64_t)a, (uint64_t)b) : 0.0;
      double k = pair_key(rc, (int)ia.size(), (int)ib.size(), alpha, tau, u);
      if (!have || k < bk || (k == bk && (a < ba || (a == ba && b < bb)))) {
        have = true;
        bk = k;
        ba = a;
        bb = b;
      }
    }
    if (!have) {
      auto it = live.begin();
      ba = it->first;
      ++it;
      bb = it->first;
    }
    IdSet nw = set_xor(live[ba], live[bb]);
    for (int32_t x : set_or(live[ba], live[bb])) {
      auto& o = owner[x];
      o.erase(std::remove_if(o.begin(), o.end(), [&](int32_t u) { return u == ba || u == bb; }),
              o.end());
      if (set_has(nw, x))
        o.push_back(nxt);
      else if (o.empty())
        owner.erase(x);
    }
    live.erase(ba);
    live.erase(bb);
    live[nxt] = nw;
    path.push_back(ba);
    path.push_back(bb);
    ++nxt;
    ++step;
  }
  return path;
}

Tree Tree::build(const std::vector<IdSet>& leaves, const int32_t* path) {
  Tree t;
  t.L = (int32_t)leaves.size();
  t.sets = leaves;
  t.kids.assign(t.L, {-1, -1});
  int32_t n = 2 * t.L - 1;
  t.parent.assign(n, -1);
  std::vector<char> used(n, 0);
  for (int32_t k = 0; k + 1 < t.L; ++k) {
    int32_t a = path[2 * k], b = path[2 * k + 1], v = t.L + k;
    require(a >= 0 && b >= 0 && a < v && b < v && a != b,
            "path step " + std::to_string(k) + " names an invalid SSA id");
    require(!used[a] && !used[b], "path step " + std::to_string(k) + " reuses a consumed tensor");
    used[a] = used[b] = 1;
    t.sets.push_back(set_xor(t.sets[a], t.sets[b]));
    t.kids.push_back({a, b});
    t.parent[a] = v;
    t.parent[b] = v;
  }
  return t;
}

BigSum Tree::cost() const {
  BigSum s;
  for (int32_t v = L; v < (int32_t)sets.size(); ++v) s.add_pow2((int)node_set(v).size());
  return s;
}

BigSum Tree::sliced_cost(const IdSet& S) const {
  BigSum s;
  for (int32_t v = L; v < (int32_t)sets.size(); ++v) {
    IdSet sv = node_set(v);
    int e = (int)sv.size() + (int)S.size() - (int)set_and(S, sv).size();
    s.add_pow2(e);
  }
  return s;
}

int Tree::space(const IdSet& S) const {
  int m = 0;
  for (auto& s : sets) m = std::max(m, (int)set_minus(s, S).size());
  return m;
}

static void big_add(BigSum& a, const BigSum& b) {
  if (a.w.size() < b.w.size()) a.w.resize(b.w.size(), 0);
  uint64_t carry = 0;
  for (size_t i = 0; i < a.w.size(); ++i) {
    uint64_t bi = i < b.w.size() ? b.w[i] : 0;
    uint64_t s = a.w[i] + bi;
    uint64_t c1 = s < a.w[i];
    uint64_t s2 = s + carry;
    uint64_t c2 = s2 < s;
    a.w[i] = s2;
    carry = c1 | c2;
  }
  if (carry) a.w.push_back(1);
}

std::vector<int32_t> Tree::stem() const {
  int32_t n = (int32_t)sets.size();
  std::vector<BigSum> best(n), sub(n);
  for (int32_t v = L; v < n; ++v) {
    auto [a, b] = kids[v];
    BigSum c;
    c.add_pow2((int)node_set(v).size());
    BigSum bv = c;
    big_add(bv, best[a].compare(best[b]) >= 0 ? best[a] : best[b]);
    best[v] = bv;
    BigSum sv = c;
    big_add(sv, sub[a]);
    big_add(sv, sub[b]);
    sub[v] = sv;
  }
  std::vector<int32_t> out{root()};
  int32_t v = root();
  while (v >= L) {
    auto [a, b] = kids[v];
    // larger best, then larger subtree cost, then smaller id
    int c = best[a].compare(best[b]);
    if (c == 0) c = sub[a].compare(sub[b]);
    int32_t pick = c > 0 ? a : (c < 0 ? b : std::min(a, b));
    out.push_back(pick);
    v = pick;
  }
  std::reverse(out.begin(), out.end());
  return out;
}

// Lifetime-based slice finder (Sec. 4.2, Algorithm 1). The lifetime of an
// index on the stem is one interval of stem positions (Linearity theorem:
// the tensors holding an index form one path of the tree, which meets the
// stem in one stretch). The over-cap stem tensors are fixed from the ends
// inwards: the end of smaller rank (root side on a tie) gets as many of its
// unsliced indices sliced as it exceeds t by, those whose interval covers
// the most over-cap tensors first (then the most tree tensors holding the
// index, then the smaller id). Off-stem tensors still above t are fixed
// afterwards in id order by their index held by the most tree tensors.
std::vector<int32_t> slice_finder(const std::vector<IdSet>& leaves, const int32_t* path, int t,
                                  const std::vector<int32_t>& pre) {
  std::vector<int32_t> S(pre.begin(), pre.end());
  if (t < 0) return S;
  IdSet ps(pre.begin(), pre.end());
  std::sort(ps.begin(), ps.end());
  std::vector<IdSet> lv(leaves.size());
  for (size_t i = 0; i < leaves.size(); ++i) lv[i] = set_minus(leaves[i], ps);
  Tree tree = Tree::build(lv, path);
  const int32_t n = (int32_t)tree.sets.size();
  std::unordered_map<int32_t, int> whole;
  for (auto& s : tree.sets)
    for (int32_t x : s) whole[x]++;
  IdSet inS;  // sorted, the indices added here
  auto rank = [&](int32_t v) { return (int)set_minus(tree.sets[v], inS).size(); };
  auto add = [&](int32_t x) {
    S.push_back(x);
    inS.insert(std::lower_bound(inS.begin(), inS.end(), x), x);
  };
  const std::vector<int32_t> stem = tree.stem();
  std::unordered_map<int32_t, std::pair<int, int>> iv;  // index -> [first, last] stem position
  for (int p = 0; p < (int)stem.size(); ++p)
    for (int32_t x : tree.sets[stem[p]]) {
      auto it = iv.find(x);
      if (it == iv.end()) iv.emplace(x, std::make_pair(p, p));
      else it->second.second = p;
    }
  std::vector<int> over;  // stem positions still above t, leaf side first
  auto trim = [&]() {
    std::vector<int> keep;
    for (int p : over)
      if (rank(stem[p]) > t) keep.push_back(p);
    over.swap(keep);
  };
  for (int p = 0; p < (int)stem.size(); ++p) over.push_back(p);
  trim();
  while (!over.empty()) {
    const int p = rank(stem[over.front()]) < rank(stem[over.back()]) ? over.front() : over.back();
    const int32_t v = stem[p];
    IdSet cand = set_minus(tree.sets[v], inS);
    std::unordered_map<int32_t, int> span;
    for (int32_t x : cand) {
      auto [lo, hi] = iv[x];
      span[x] = (int)(std::upper_bound(over.begin(), over.end(), hi) -
                      std::lower_bound(over.begin(), over.end(), lo));
    }
    std::sort(cand.begin(), cand.end(), [&](int32_t x, int32_t y) {
      if (span[x] != span[y]) return span[x] > span[y];
      if (whole[x] != whole[y]) return whole[x] > whole[y];
      return x < y;
    });
    const int need = rank(v) - t;
    for (int i = 0; i < need; ++i) add(cand[i]);
    trim();
  }
  for (int32_t v = 0; v < n; ++v) {
    while (rank(v) > t) {
      IdSet cand = set_minus(tree.sets[v], inS);
      int32_t best = cand[0];
      for (int32_t x : cand)
        if (whole[x] > whole[best] || (whole[x] == whole[best] && x < best)) best = x;
      add(best);
    }
  }
  return S;
}

// a - b for a >= b
static BigSum big_sub(const BigSum& a, const BigSum& b) {
  BigSum r = a;
  uint64_t borrow = 0;
  for (size_t i = 0; i < r.w.size(); ++i) {
    uint64_t bi = i < b.w.size() ? b.w[i] : 0;
    uint64_t d = r.w[i] - bi;
    uint64_t b1 = r.w[i] < bi;
    uint64_t d2 = d - borrow;
    uint64_t b2 = d < borrow;
    r.w[i] = d2;
    borrow = b1 | b2;
  }
  while (!r.w.empty() && r.w.back() == 0) r.w.pop_back();
  return r;
}

namespace {

// Eq. (4) for a slicing set and its one-element variants. Each contraction
// node keeps |S n s_v|; a variant that removes `out` (or nothing, -1) and
// adds `in` (or nothing) changes it by membership only.
struct SlicedCost {
  const Tree& tree;
  std::vector<IdSet> ns;    // s_v of every contraction node
  std::vector<int> inter;   // |S n s_v| for the current S
  int nS = 0;
  explicit SlicedCost(const Tree& t) : tree(t) {
    for (int32_t v = t.L; v < (int32_t)t.sets.size(); ++v) ns.push_back(t.node_set(v));
    inter.assign(ns.size(), 0);
  }
  void reset(const std::vector<int32_t>& S) {
    IdSet s(S.begin(), S.end());
    std::sort(s.begin(), s.end());
    nS = (int)s.size();
    for (size_t v = 0; v < ns.size(); ++v) inter[v] = (int)set_and(ns[v], s).size();
  }
  BigSum variant(int32_t out, int32_t in) const {
    BigSum c;
    int n = nS - (out >= 0) + (in >= 0);
    for (size_t v = 0; v < ns.size(); ++v) {
      int k = inter[v];
      if (out >= 0 && set_has(ns[v], out)) --k;
      if (in >= 0 && set_has(ns[v], in)) ++k;
      c.add_pow2((int)ns[v].size() + n - k);
    }
    return c;
  }
};

int dim_after(const IdSet& s, const std::vector<char>& inS) {
  int d = 0;
  for (int32_t x : s) d += !inS[x];
  return d;
}

}  // namespace

std::vector<int32_t> slice_refine(const Tree& tree, int t, const std::vector<int32_t>& S0,
                                  const RefineParams& p, RefineStats* st) {
  int32_t max_id = -1;
  for (auto& s : tree.sets)
    for (int32_t x : s) max_id = std::max(max_id, x);
  for (int32_t x : S0) max_id = std::max(max_id, x);
  std::vector<char> inS(max_id + 1, 0);
  for (int32_t x : S0) {
    require(x >= 0 && !inS[x], "slicing set has a negative or repeated id");
    inS[x] = 1;
  }
  for (auto& s : tree.sets)
    require(dim_after(s, inS) <= t, "the slicing set does not meet the target rank", LTN_E_CAP);
  require(p.n_fixed >= 0 && p.n_fixed <= (int)S0.size(), "n_fixed out of range");
  require(p.iters_per_temp >= 1, "iters_per_temp must be >= 1");
  require(p.alpha > 0.0 && p.alpha < 1.0, "alpha must be in (0, 1)");
  require(p.tf > 0.0 && p.t0 > 0.0, "temperatures must be positive");
  // lifetime of every index: the tree tensors holding it, ascending id
  std::vector<std::vector<int32_t>> life(max_id + 1);
  for (int32_t v = 0; v < (int32_t)tree.sets.size(); ++v)
    for (int32_t x : tree.sets[v]) life[x].push_back(v);
  RefineStats stats;
  std::vector<int32_t> cur = S0;
  SlicedCost sc(tree);
  sc.reset(cur);
  BigSum cur_c = sc.variant(-1, -1);
  std::vector<int32_t> best = cur;
  BigSum best_c = cur_c;
  double T = p.t0;
  int64_t it = 0;
  for (;;) {
    for (int r = 0; r < p.iters_per_temp; ++r) {
      const int free = (int)cur.size() - p.n_fixed;
      if (free <= 0) break;
      const double u = keyed_uniform(p.seed, (uint64_t)it, 0, 0);
      const int slot = p.n_fixed + std::min((int)(u * free), free - 1);
      const int32_t idx = cur[slot];
      // critical tensors of idx (Algorithm 3): its lifetime at rank t
      std::vector<int32_t> crit;
      for (int32_t v : life[idx])
        if (dim_after(tree.sets[v], inS) == t) crit.push_back(v);
      if (crit.empty()) {
        inS[idx] = 0;
        cur.erase(cur.begin() + slot);
        sc.reset(cur);
        cur_c = sc.variant(-1, -1);
        ++stats.dropped;
      } else {
        // replacements (Algorithm 4): unsliced indices whose lifetime
        // contains every critical tensor; each holds crit[0], so only its
        // indices need checking
        IdSet c2;
        for (int32_t x : tree.sets[crit[0]]) {
          if (inS[x]) continue;
          bool all = true;
          for (int32_t v : crit)
            if (!std::binary_search(life[x].begin(), life[x].end(), v)) { all = false; break; }
          if (all) c2.push_back(x);
        }
        for (int32_t c : c2) {
          const int32_t occupant = cur[slot];
          BigSum new_c = sc.variant(occupant, c);
          ++stats.proposals;
          bool take;
          if (new_c.compare(cur_c) < 0) {
            take = true;
          } else {
            const double rel = big_sub(new_c, cur_c).to_double() / cur_c.to_double();
            const double prob = std::exp(-rel / T);
            take = keyed_uniform(p.seed, (uint64_t)it, 1, (uint64_t)c) < prob;
          }
          if (take) {
            inS[occupant] = 0;
            inS[c] = 1;
            cur[slot] = c;
            sc.reset(cur);
            cur_c = new_c;
            ++stats.accepted;
          }
          if (cur_c.compare(best_c) < 0) {
            best = cur;
            best_c = cur_c;
          }
        }
      }
      if (cur_c.compare(best_c) < 0) {
        best = cur;
        best_c = cur_c;
      }
      ++it;
    }
    stats.iterations = (int32_t)it;
    T = T * p.alpha;
    if (T < p.tf || (int)cur.size() <= p.n_fixed) break;
  }
  if (st) *st = stats;
  return best;
}

// Subtree reconfiguration. Node costs 2^|s_v - S| as 128-bit integers that
// saturate at 2^120; a sweep visits every contraction node once (ids of the
// tree at the start of the sweep), then the tree is written out again in
// post order.
namespace {
using u128 = unsigned __int128;
const u128 kSat = (u128)1 << 120;
inline u128 sat(u128 x) { return x < kSat ? x : kSat; }
inline u128 pow2_sat(int e) { return e < 120 ? ((u128)1 << e) : kSat; }
}  // namespace

std::vector<int32_t> reconfigure(const std::vector<IdSet>& leaves, const std::vector<int32_t>& path,
                                 int k, int sweeps, const IdSet& S, int t) {
  require(k >= 2 && k <= 16, "subtree size k must be in 2..16");
  const int32_t L = (int32_t)leaves.size();
  const int32_t n = L + (int32_t)path.size() / 2;
  std::vector<IdSet> sets(leaves.begin(), leaves.end());
  std::vector<std::pair<int32_t, int32_t>> kids(L, {-1, -1});
  for (size_t s = 0; s + 1 < path.size(); s += 2) {
    sets.push_back(set_xor(sets[path[s]], sets[path[s + 1]]));
    kids.push_back({path[s], path[s + 1]});
  }
  auto unsliced = [&](const IdSet& x) { return (int)set_minus(x, S).size(); };
  auto node_cost = [&](const IdSet& a, const IdSet& b) { return pow2_sat(unsliced(set_or(a, b))); };
  std::vector<int32_t> out_path(path);
  for (int sw = 0; sw < sweeps; ++sw) {
    bool improved = false;
    for (int32_t v = L; v < n; ++v) {
      std::vector<int32_t> front{v};
      while ((int)front.size() < k) {
        int32_t pick = -1;
        int psz = -1;
        for (int32_t u : front) {
          if (kids[u].first < 0) continue;
          int sz = unsliced(set_or(sets[kids[u].first], sets[kids[u].second]));
          if (sz > psz || (sz == psz && u < pick)) {
            psz = sz;
            pick = u;
          }
        }
        if (pick < 0) break;
        front.erase(std::find(front.begin(), front.end(), pick));
        front.push_back(kids[pick].first);
        front.push_back(kids[pick].second);
      }
      const int m = (int)front.size();
      if (m < 3) continue;
      // inner nodes in pre order (node, left subtree, right subtree)
      std::vector<int32_t> inner;
      std::vector<int32_t> stack{v};
      while (!stack.empty()) {
        int32_t u = stack.back();
        stack.pop_back();
        if (std::find(front.begin(), front.end(), u) != front.end()) continue;
        inner.push_back(u);
        stack.push_back(kids[u].second);
        stack.push_back(kids[u].first);
      }
      u128 old = 0;
      for (int32_t u : inner) old = sat(old + node_cost(sets[kids[u].first], sets[kids[u].second]));
      if (old >= kSat) continue;
      const uint32_t full = (1u << m) - 1;
      // frontier tensors without S as bit sets over their local index universe
      IdSet uni;
      for (int32_t u : front) uni = set_or(uni, set_minus(sets[u], S));
      const int W = std::max<int>(1, ((int)uni.size() + 63) / 64);
      std::vector<uint64_t> tens((size_t)(full + 1) * W, 0);
      for (int i = 0; i < m; ++i) {
        uint64_t* dst = &tens[(size_t)(1u << i) * W];
        for (int32_t x : set_minus(sets[front[i]], S)) {
          int pos = (int)(std::lower_bound(uni.begin(), uni.end(), x) - uni.begin());
          dst[pos / 64] |= 1ull << (pos % 64);
        }
      }
      for (uint32_t M = 1; M <= full; ++M) {
        uint32_t low = M & (~M + 1);
        if (low == M) continue;
        const uint64_t* a = &tens[(size_t)(M ^ low) * W];
        const uint64_t* b = &tens[(size_t)low * W];
        uint64_t* d = &tens[(size_t)M * W];
        for (int j = 0; j < W; ++j) d[j] = a[j] ^ b[j];
      }
      auto rank_of = [&](uint32_t M) {
        int r = 0;
        const uint64_t* a = &tens[(size_t)M * W];
        for (int j = 0; j < W; ++j) r += __builtin_popcountll(a[j]);
        return r;
      };
      auto union_rank = [&](uint32_t A, uint32_t B) {
        int r = 0;
        const uint64_t* a = &tens[(size_t)A * W];
        const uint64_t* b = &tens[(size_t)B * W];
        for (int j = 0; j < W; ++j) r += __builtin_popcountll(a[j] | b[j]);
        return r;
      };
      std::vector<u128> best(full + 1, 0);
      std::vector<uint32_t> choice(full + 1, 0);
      for (uint32_t M = 1; M <= full; ++M) {
        if ((M & (M - 1)) == 0) continue;
        if (t >= 0 && M != full && rank_of(M) > t) {
          best[M] = kSat;
          continue;
        }
        bool have = false;
        u128 bc = 0;
        uint32_t bsub = 0;
        for (uint32_t sub = (M - 1) & M; sub; sub = (sub - 1) & M) {
          uint32_t o = M ^ sub;
          if (sub >= o) continue;
          u128 c = sat(sat(best[sub] + best[o]) + pow2_sat(union_rank(sub, o)));
          if (!have || c < bc) {
            have = true;
            bc = c;
            bsub = sub;
          }
        }
        best[M] = bc;
        choice[M] = bsub;
      }
      if (best[full] >= old) continue;
      improved = true;
      std::vector<int32_t> pool;
      for (int32_t u : inner)
        if (u != v) pool.push_back(u);
      // rebuild in post order: children first, new ids taken from the end of the pool
      std::function<int32_t(uint32_t, bool)> assign = [&](uint32_t M, bool root) -> int32_t {
        if ((M & (M - 1)) == 0) return front[__builtin_ctz(M)];
        int32_t a = assign(choice[M], false);
        int32_t b = assign(M ^ choice[M], false);
        int32_t u = v;
        if (!root) {
          u = pool.back();
          pool.pop_back();
        }
        kids[u] = {a, b};
        sets[u] = set_xor(sets[a], sets[b]);
        return u;
      };
      assign(full, true);
    }
    // post order from the root, left child first
    std::vector<int32_t> order;
    std::vector<std::pair<int32_t, bool>> st{{n - 1, false}};
    while (!st.empty()) {
      auto [u, done] = st.back();
      st.pop_back();
      if (kids[u].first < 0) continue;
      if (done) {
        order.push_back(u);
      } else {
        st.push_back({u, true});
        st.push_back({kids[u].second, false});
        st.push_back({kids[u].first, false});
      }
    }
    std::vector<int32_t> newid(n, 0);
    for (int32_t i = 0; i < L; ++i) newid[i] = i;
    out_path.clear();
    for (int32_t u : order) {
      newid[u] = L + (int32_t)out_path.size() / 2;
      out_path.push_back(newid[kids[u].first]);
      out_path.push_back(newid[kids[u].second]);
    }
    sets.resize(L);
    kids.resize(L);
    for (size_t s = 0; s + 1 < out_path.size(); s += 2) {
      sets.push_back(set_xor(sets[out_path[s]], sets[out_path[s + 1]]));
      kids.push_back({out_path[s], out_path[s + 1]});
    }
    if (!improved) break;
  }
  return out_path;
}

std::vector<int32_t> slice_greedy_overhead(const Tree& tree, int t, const std::vector<int32_t>& pre) {
  std::vector<int32_t> S = pre;
  if (t < 0) return S;
  int32_t max_id = -1;
  for (auto& s : tree.sets)
    for (int32_t x : s) max_id = std::max(max_id, x);
  for (int32_t x : pre) max_id = std::max(max_id, x);
  std::vector<char> inS(max_id + 1, 0);
  for (int32_t x : pre) inS[x] = 1;
  SlicedCost sc(tree);
  for (;;) {
    std::map<int32_t, int> count;  // ascending id
    for (auto& s : tree.sets)
      if (dim_after(s, inS) > t)
        for (int32_t x : s)
          if (!inS[x]) count[x]++;
    if (count.empty()) return S;
    sc.reset(S);
    bool have = false;
    BigSum bc;
    int32_t pick = -1;
    for (auto [x, n] : count) {
      BigSum c = sc.variant(-1, x);
      int cmp = have ? c.compare(bc) : -1;
      if (!have || cmp < 0 || (cmp == 0 && n > count[pick])) {
        have = true;
        bc = c;
        pick = x;
      }
    }
    S.push_back(pick);
    inS[pick] = 1;
  }
}

}  // namespace ltn

using namespace ltn;

extern "C" ltn_status ltn_greedy_path(const ltn_network* net, const int32_t* exclude,
                                      int32_t n_exclude, double alpha, double tau, uint64_t seed,
                                      int32_t* path_out) {
  return guarded([&] {
    Net n = Net::from_abi(net, false);
    require(path_out != nullptr, "path_out is NULL");
    require(n_exclude >= 0 && (n_exclude == 0 || exclude), "bad exclude list");
    IdSet ex(exclude, exclude + n_exclude);
    std::sort(ex.begin(), ex.end());
    auto p = greedy(n.sets, ex, alpha, tau, seed);
    std::copy(p.begin(), p.end(), path_out);
  });
}

extern "C" ltn_status ltn_tree_costs(const ltn_network* net, const int32_t* path, const int32_t* S,
                                     int32_t n_sliced, ltn_costs* out) {
  return guarded([&] {
    Net n = Net::from_abi(net, false);
    require(path && out, "NULL argument");
    require(n_sliced >= 0 && (n_sliced == 0 || S), "bad slicing set");
    Tree t = Tree::build(n.sets, path);
    IdSet s(S, S + n_sliced);
    std::sort(s.begin(), s.end());
    BigSum c = t.cost(), cs = t.sliced_cost(s);
    out->log2_cost = c.log2();
    out->log2_sliced = cs.log2();
    out->overhead = std::exp2(out->log2_sliced - out->log2_cost);
    out->space_log2 = t.space(s);
    out->space_log2_unsliced = t.space({});
    c.to_words(out->cost_words, 4);
    cs.to_words(out->sliced_words, 4);
    out->stem_len = (int32_t)t.stem().size();
  });
}

extern "C" ltn_status ltn_tree_stem(const ltn_network* net, const int32_t* path, int32_t* stem_out,
                                    int32_t cap, int32_t* len) {
  return guarded([&] {
    Net n = Net::from_abi(net, false);
    require(path && stem_out && len, "NULL argument");
    auto st = Tree::build(n.sets, path).stem();
    require((int32_t)st.size() <= cap, "stem_out too small", LTN_E_NOMEM);
    std::copy(st.begin(), st.end(), stem_out);
    *len = (int32_t)st.size();
  });
}

extern "C" ltn_status ltn_stem_profile(const ltn_network* net, const int32_t* path, const int32_t* S,
                                       int32_t n_sliced, ltn_stem_row* rows, int32_t cap, int32_t* len) {
  return guarded([&] {
    Net n = Net::from_abi(net, false);
    require(path && rows && len, "NULL argument");
    require(n_sliced == 0 || S != nullptr, "S is NULL");
    IdSet sl(S, S + n_sliced);
    std::sort(sl.begin(), sl.end());
    Tree tree = Tree::build(n.sets, path);
    auto st = tree.stem();
    require((int32_t)st.size() <= cap, "rows too small", LTN_E_NOMEM);
    for (size_t i = 0; i < st.size(); ++i) {
      const int32_t v = st[i];
      ltn_stem_row& r = rows[i];
      r.tensor = v;
      r.rank = (int32_t)tree.sets[v].size();
      r.rank_sliced = (int32_t)set_minus(tree.sets[v], sl).size();
      if (v < tree.L) {
        r.node_bits = r.node_bits_sliced = -1;
      } else {
        const IdSet ns = tree.node_set(v);
        r.node_bits = (int32_t)ns.size();
        r.node_bits_sliced = (int32_t)set_minus(ns, sl).size();
      }
    }
    *len = (int32_t)st.size();
  });
}

extern "C" ltn_status ltn_slice_finder(const ltn_network* net, const int32_t* path, int32_t t,
                                       const int32_t* pre, int32_t n_pre, int32_t* S_out,
                                       int32_t cap, int32_t* n_sliced) {
  return guarded([&] {
    Net n = Net::from_abi(net, false);
    require(path && S_out && n_sliced, "NULL argument");
    require(n_pre >= 0 && (n_pre == 0 || pre), "bad pre list");
    std::vector<int32_t> p(pre, pre + n_pre);
    auto S = slice_finder(n.sets, path, t, p);
    require((int32_t)S.size() <= cap, "S_out too small", LTN_E_NOMEM);
    std::copy(S.begin(), S.end(), S_out);
    *n_sliced = (int32_t)S.size();
  });
}

extern "C" ltn_status ltn_path_search(const ltn_network* net, int32_t t, const int32_t* pre,
                                      int32_t n_pre, const ltn_search_opts* o, int32_t* path_out,
                                      int32_t* S_out, int32_t cap, int32_t* n_sliced,
                                      int32_t* best_trial) {
  return guarded([&] {
    Net n = Net::from_abi(net, false);
    require(o && path_out && S_out && n_sliced, "NULL argument");
    require(o->n_alpha >= 1 && o->alphas && o->n_tau >= 1 && o->taus && o->n_seeds >= 1,
            "empty search grid");
    require(n_pre >= 0 && (n_pre == 0 || pre), "bad pre list");
    require(o->reconf_k == 0 || (o->reconf_k >= 3 && o->reconf_k <= 16 && o->reconf_sweeps >= 0),
            "reconf_k must be 0 or in 3..16, reconf_sweeps >= 0");
    std::vector<int32_t> p(pre, pre + n_pre);
    IdSet ex(p.begin(), p.end());
    std::sort(ex.begin(), ex.end());
    bool have = false;
    BigSum bc;
    size_t bs = 0;
    int32_t btrial = -1, trial = 0;
    std::vector<int32_t> bpath, bS;
    for (int ia = 0; ia < o->n_alpha; ++ia)
      for (int it = 0; it < o->n_tau; ++it) {
        int seeds = o->taus[it] > 0.0 ? o->n_seeds : 1;
        for (int sd = 0; sd < seeds; ++sd, ++trial) {
          auto path = greedy(n.sets, ex, o->alphas[ia], o->taus[it], o->seed_base + (uint64_t)sd);
          if (o->reconf_k >= 3) path = reconfigure(n.sets, path, o->reconf_k, o->reconf_sweeps, ex, -1);
          auto S = slice_finder(n.sets, path.data(), t, p);
          if (o->reconf_k >= 3 && t >= 0) {
            IdSet ss(S.begin(), S.end());
            std::sort(ss.begin(), ss.end());
            path = reconfigure(n.sets, path, o->reconf_k, o->reconf_sweeps, ss, t);
          }
          Tree tr = Tree::build(n.sets, path.data());
          IdSet ss(S.begin(), S.end());
          std::sort(ss.begin(), ss.end());
          BigSum c = tr.sliced_cost(ss);
          int cmp = have ? c.compare(bc) : -1;
          if (!have || cmp < 0 || (cmp == 0 && S.size() < bs)) {
            have = true;
            bc = c;
            bs = S.size();
            btrial = trial;
            bpath = path;
            bS = S;
          }
        }
      }
    require((int32_t)bS.size() <= cap, "S_out too small", LTN_E_NOMEM);
    std::copy(bpath.begin(), bpath.end(), path_out);
    std::copy(bS.begin(), bS.end(), S_out);
    *n_sliced = (int32_t)bS.size();
    if (best_trial) *best_trial = btrial;
  });
}

extern "C" ltn_status ltn_slice_refine(const ltn_network* net, const int32_t* path, int32_t t,
                                       const int32_t* S_in, int32_t n_in,
                                       const ltn_refine_opts* o, int32_t* S_out, int32_t* n_out,
                                       ltn_refine_stats* stats) {
  return guarded([&] {
    Net n = Net::from_abi(net, false);
    require(path && o && S_out && n_out, "NULL argument");
    require(t >= 0, "the refiner needs a target rank t >= 0");
    require(n_in >= 0 && (n_in == 0 || S_in), "bad slicing set");
    Tree tr = Tree::build(n.sets, path);
    RefineParams rp;
    rp.t0 = o->t0;
    rp.alpha = o->alpha;
    rp.tf = o->tf;
    rp.iters_per_temp = o->iters_per_temp;
    rp.n_fixed = o->n_fixed;
    rp.seed = o->seed;
    RefineStats st;
    auto S = slice_refine(tr, t, std::vector<int32_t>(S_in, S_in + n_in), rp, &st);
    std::copy(S.begin(), S.end(), S_out);
    *n_out = (int32_t)S.size();
    if (stats) {
      stats->iterations = st.iterations;
      stats->proposals = st.proposals;
      stats->accepted = st.accepted;
      stats->dropped = st.dropped;
    }
  });
}

extern "C" ltn_status ltn_slice_greedy_overhead(const ltn_network* net, const int32_t* path,
                                                int32_t t, const int32_t* pre, int32_t n_pre,
                                                int32_t* S_out, int32_t cap, int32_t* n_sliced) {
  return guarded([&] {
    Net n = Net::from_abi(net, false);
    require(path && S_out && n_sliced, "NULL argument");
    require(n_pre >= 0 && (n_pre == 0 || pre), "bad pre list");
    Tree tr = Tree::build(n.sets, path);
    auto S = slice_greedy_overhead(tr, t, std::vector<int32_t>(pre, pre + n_pre));
    require((int32_t)S.size() <= cap, "S_out too small", LTN_E_NOMEM);
    std::copy(S.begin(), S.end(), S_out);
    *n_sliced = (int32_t)S.size();
  });
}

extern "C" ltn_status ltn_tree_reconfigure(const ltn_network* net, const int32_t* path, int32_t k,
                                           int32_t sweeps, const int32_t* S, int32_t n_sliced,
                                           int32_t t, int32_t* path_out) {
  return guarded([&] {
    Net n = Net::from_abi(net, false);
    require(path && path_out, "NULL argument");
    require(sweeps >= 0, "sweeps must be >= 0");
    require(n_sliced >= 0 && (n_sliced == 0 || S), "bad slicing set");
    const int32_t L = (int32_t)n.sets.size();
    Tree::build(n.sets, path);  // validates the SSA path
    IdSet s(S, S + n_sliced);
    std::sort(s.begin(), s.end());
    std::vector<int32_t> p(path, path + 2 * std::max(0, L - 1));
    auto r = reconfigure(n.sets, p, k, sweeps, s, t);
    std::copy(r.begin(), r.end(), path_out);
  });
}
