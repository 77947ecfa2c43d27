// Internal helpers of libltn: error reporting, exact power-of-two sums and
// bit utilities. Not part of the public ABI.
#pragma once

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>
#include <stdexcept>

#include "ltn.h"

namespace ltn {

// Thrown inside the library, turned into a status + message at the ABI.
struct Error : std::runtime_error {
  ltn_status code;
  Error(ltn_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

template <typename F>
ltn_status guarded(F&& f) {
  try {
    f();
    return LTN_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return LTN_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return LTN_E_INVALID;
  }
}

[[noreturn]] inline void fail(ltn_status c, const std::string& m) { throw Error(c, m); }
inline void require(bool ok, const std::string& m, ltn_status c = LTN_E_INVALID) {
  if (!ok) fail(c, m);
}

// Exact non-negative integer as little-endian 64-bit words; only sums of
// powers of two are needed (Eq. (1) and Eq. (4) are such sums).
struct BigSum {
  std::vector<uint64_t> w;
  void add_pow2(int e) {
    size_t word = (size_t)e / 64;
    if (w.size() <= word) w.resize(word + 1, 0);
    uint64_t bit = 1ull << (e % 64);
    for (size_t i = word;; ++i) {
      if (i == w.size()) w.push_back(0);
      uint64_t old = w[i];
      w[i] = old + bit;
      if (w[i] >= old) break;  // no carry
      bit = 1;
    }
  }
  int compare(const BigSum& o) const {
    size_t n = std::max(w.size(), o.w.size());
    for (size_t i = n; i-- > 0;) {
      uint64_t a = i < w.size() ? w[i] : 0, b = i < o.w.size() ? o.w[i] : 0;
      if (a != b) return a < b ? -1 : 1;
    }
    return 0;
  }
  double log2() const;
  double to_double() const;  // correctly rounded, ties to even
  void to_words(uint64_t* out, int n) const {
    for (int i = 0; i < n; ++i) out[i] = i < (int)w.size() ? w[i] : 0;
  }
};

// Sorted small set of index ids.
using IdSet = std::vector<int32_t>;
IdSet set_xor(const IdSet& a, const IdSet& b);
IdSet set_or(const IdSet& a, const IdSet& b);
IdSet set_and(const IdSet& a, const IdSet& b);
IdSet set_minus(const IdSet& a, const IdSet& b);
bool set_has(const IdSet& a, int32_t x);

// The network as plain C++ vectors (copied from an ltn_network).
struct Net {
  std::vector<IdSet> axes;   // per leaf, axis order as given (not sorted)
  std::vector<IdSet> sets;   // per leaf, sorted
  std::vector<int32_t> open_ids;
  std::vector<int32_t> param;
  std::vector<int64_t> data_off;  // element offset of each leaf's data
  int32_t n_indices = 0;
  static Net from_abi(const ltn_network* net, bool check);
};

// Contraction tree of an SSA path (Sec. 2.1.1): node v < L is a leaf,
// node L+k is the k-th contraction.
struct Tree {
  int32_t L = 0;
  std::vector<IdSet> sets;                    // tensor of every node
  std::vector<std::pair<int32_t, int32_t>> kids;
  std::vector<int32_t> parent;
  int32_t root() const { return (int32_t)sets.size() - 1; }
  static Tree build(const std::vector<IdSet>& leaves, const int32_t* path);
  IdSet node_set(int32_t v) const { return set_or(sets[kids[v].first], sets[kids[v].second]); }
  BigSum cost() const;                        // Eq. (1)
  BigSum sliced_cost(const IdSet& S) const;   // Eq. (4)
  int space(const IdSet& S) const;            // log2 of the largest tensor
  std::vector<int32_t> stem() const;
};

std::vector<int32_t> greedy(const std::vector<IdSet>& leaves, const IdSet& exclude, double alpha,
                            double tau, uint64_t seed);
std::vector<int32_t> slice_finder(const std::vector<IdSet>& leaves, const int32_t* path, int t,
                                  const std::vector<int32_t>& pre);

struct RefineParams {
  double t0 = 1.0, alpha = 0.98, tf = 1e-3;
  int iters_per_temp = 1, n_fixed = 0;
  uint64_t seed = 0;
};
struct RefineStats {
  int32_t iterations = 0, proposals = 0, accepted = 0, dropped = 0;
};
std::vector<int32_t> slice_refine(const Tree& tree, int t, const std::vector<int32_t>& S,
                                  const RefineParams& p, RefineStats* st);
std::vector<int32_t> reconfigure(const std::vector<IdSet>& leaves, const std::vector<int32_t>& path,
                                 int k, int sweeps, const IdSet& S, int t);
std::vector<int32_t> slice_greedy_overhead(const Tree& tree, int t, const std::vector<int32_t>& pre);

}  // namespace ltn
