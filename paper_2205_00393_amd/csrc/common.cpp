#include "common.h"

#include <algorithm>
#include <cmath>

namespace ltn {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

double BigSum::log2() const {
  // value = sum w[i] 2^(64 i); enough precision from the top two words
  for (size_t i = w.size(); i-- > 0;) {
    if (w[i] == 0) continue;
    double hi = (double)w[i];
    double lo = i > 0 ? (double)w[i - 1] / 18446744073709551616.0 : 0.0;
    return std::log2(hi + lo) + 64.0 * (double)i;
  }
  return -INFINITY;
}

double BigSum::to_double() const {
  int top = -1;
  for (size_t i = w.size(); i-- > 0;)
    if (w[i]) {
      top = (int)i * 64 + 63 - __builtin_clzll(w[i]);
      break;
    }
  if (top < 0) return 0.0;
  if (top < 53) return (double)w[0];  // exact
  auto bit = [&](int i) -> uint64_t { return (w[(size_t)i / 64] >> (i % 64)) & 1; };
  const int low = top - 52;  // weight of the last kept bit
  uint64_t m = 0;
  for (int i = top; i >= low; --i) m = (m << 1) | bit(i);
  const bool half = bit(low - 1) != 0;
  bool sticky = false;
  for (int i = low - 2; i >= 0 && !sticky; --i) sticky = bit(i) != 0;
  if (half && (sticky || (m & 1))) ++m;
  return std::ldexp((double)m, low);
}

IdSet set_xor(const IdSet& a, const IdSet& b) {
  IdSet r;
  std::set_symmetric_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}
IdSet set_or(const IdSet& a, const IdSet& b) {
  IdSet r;
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}
IdSet set_and(const IdSet& a, const IdSet& b) {
  IdSet r;
  std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}
IdSet set_minus(const IdSet& a, const IdSet& b) {
  IdSet r;
  std::set_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}
bool set_has(const IdSet& a, int32_t x) { return std::binary_search(a.begin(), a.end(), x); }

Net Net::from_abi(const ltn_network* net, bool check) {
  require(net != nullptr, "network is NULL");
  require(net->n_leaves >= 1, "network has no leaves");
  require(net->leaf_off && net->index_ids, "network arrays are NULL");
  require(net->n_indices >= 0, "negative n_indices");
  Net n;
  n.n_indices = net->n_indices;
  n.axes.resize(net->n_leaves);
  n.sets.resize(net->n_leaves);
  n.param.assign(net->n_leaves, -1);
  n.data_off.resize(net->n_leaves + 1);
  require(net->leaf_off[0] == 0, "leaf_off[0] must be 0");
  std::vector<int> count(net->n_indices, 0);
  int64_t doff = 0;
  for (int32_t i = 0; i < net->n_leaves; ++i) {
    int64_t b = net->leaf_off[i], e = net->leaf_off[i + 1];
    require(e >= b && e - b <= 62, "leaf " + std::to_string(i) + " has a bad rank");
    for (int64_t j = b; j < e; ++j) {
      int32_t x = net->index_ids[j];
      require(x >= 0 && x < net->n_indices, "leaf " + std::to_string(i) + " names unknown index " + std::to_string(x));
      n.axes[i].push_back(x);
      count[x]++;
    }
    n.sets[i] = n.axes[i];
    std::sort(n.sets[i].begin(), n.sets[i].end());
    require(std::adjacent_find(n.sets[i].begin(), n.sets[i].end()) == n.sets[i].end(),
            "leaf " + std::to_string(i) + " repeats an index");
    n.data_off[i] = doff;
    doff += int64_t(1) << (e - b);
    if (net->param_leaf) n.param[i] = net->param_leaf[i];
  }
  n.data_off[net->n_leaves] = doff;
  require(net->n_open >= 0 && (net->n_open == 0 || net->open_ids), "bad open index list");
  std::vector<char> is_open(net->n_indices, 0);
  for (int32_t j = 0; j < net->n_open; ++j) {
    int32_t x = net->open_ids[j];
    require(x >= 0 && x < net->n_indices, "unknown open index");
    require(!is_open[x], "open index listed twice");
    is_open[x] = 1;
    n.open_ids.push_back(x);
  }
  if (check) {
    for (int32_t x = 0; x < net->n_indices; ++x) {
      if (is_open[x])
        require(count[x] == 1, "open index " + std::to_string(x) + " must lie in exactly one leaf");
      else
        require(count[x] == 2 || count[x] == 0,
                "index " + std::to_string(x) + " lies in " + std::to_string(count[x]) +
                    " leaves (a closed index needs exactly two)");
    }
  }
  return n;
}

}  // namespace ltn

extern "C" const char* ltn_last_error(void) { return ltn::g_last_error.c_str(); }
extern "C" const char* ltn_version(void) { return "ltn 0.1 (gfx950)"; }
