// Circuit -> tensor network, and absorption of rank-1 / rank-2 tensors.
//
// The network of <b| C |0> has one tensor per gate (axes: outputs, then
// inputs), a |0> vector per qubit and a <b_q| vector per closed qubit; every
// wire segment is an index of size 2 (Sec. 2.1.1). Preprocessing absorbs the
// non-parameterised rank-1 and rank-2 tensors into neighbours (Sec. 2.1.2),
// which removes every single-qubit gate of a fixed-gate circuit.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>

#include "common.h"

using cd = std::complex<double>;

struct ltn_netbuf {
  std::vector<int64_t> leaf_off;
  std::vector<int32_t> index_ids;
  std::vector<float> data64;     // complex64 interleaved
  std::vector<double> data128;   // complex128 interleaved
  std::vector<int32_t> open_ids;
  std::vector<int32_t> param;
  int32_t n_indices = 0;
};

namespace {

struct T {
  std::vector<int32_t> ix;  // axes, first = slowest
  std::vector<cd> d;        // 2^rank
  int32_t param = -1;
};

std::vector<cd> gate_matrix(const ltn_gate& g) {
  const cd I(0, 1);
  auto sqrtp = [&](cd p00, cd p01, cd p10, cd p11) {
    cd a = (1.0 + I) / 2.0, b = (1.0 - I) / 2.0;
    return std::vector<cd>{a + b * p00, b * p01, b * p10, a + b * p11};
  };
  const double r2 = 1.0 / std::sqrt(2.0);
  switch (g.kind) {
    case LTN_GATE_SQRT_X: return sqrtp(0, 1, 1, 0);
    case LTN_GATE_SQRT_Y: return sqrtp(0, -I, I, 0);
    case LTN_GATE_SQRT_W: return sqrtp(0, (1.0 - I) * r2, (1.0 + I) * r2, 0);
    case LTN_GATE_FSIM: {
      double c = std::cos(g.p[0]), s = std::sin(g.p[0]);
      std::vector<cd> m(16, 0.0);
      m[0] = 1;
      m[5] = c;
      m[6] = -I * s;
      m[9] = -I * s;
      m[10] = c;
      m[15] = std::exp(-I * g.p[1]);
      return m;
    }
    case LTN_GATE_U3: {
      // Rz(a) Ry(b) Rz(c); Rz(x) = diag(e^{-ix/2}, e^{ix/2})
      cd ea = std::exp(-0.5 * I * g.p[0]), ec = std::exp(-0.5 * I * g.p[2]);
      double cb = std::cos(0.5 * g.p[1]), sb = std::sin(0.5 * g.p[1]);
      return {ea * cb * ec, -ea * sb * std::conj(ec), std::conj(ea) * sb * ec,
              std::conj(ea) * cb * std::conj(ec)};
    }
    case LTN_GATE_MATRIX: {
      int k = g.q1 >= 0 ? 2 : 1, n = (1 << k) * (1 << k);
      std::vector<cd> m(n);
      for (int i = 0; i < n; ++i) m[i] = cd(g.m[2 * i], g.m[2 * i + 1]);
      return m;
    }
  }
  ltn::fail(LTN_E_INVALID, "unknown gate kind " + std::to_string(g.kind));
}

// Contract t into n over their shared indices; result axes = n's unshared
// axes then t's unshared axes.
T merge(const T& n, const T& t) {
  std::vector<int32_t> shared;
  for (int32_t x : n.ix)
    if (std::find(t.ix.begin(), t.ix.end(), x) != t.ix.end()) shared.push_back(x);
  T r;
  for (int32_t x : n.ix)
    if (std::find(shared.begin(), shared.end(), x) == shared.end()) r.ix.push_back(x);
  for (int32_t x : t.ix)
    if (std::find(shared.begin(), shared.end(), x) == shared.end()) r.ix.push_back(x);
  r.param = n.param;
  int rn = (int)n.ix.size(), rt = (int)t.ix.size(), rr = (int)r.ix.size(), ks = (int)shared.size();
  r.d.assign(size_t(1) << rr, 0.0);
  // stride (in elements) of every index within n and t
  auto stride = [](const std::vector<int32_t>& ix, int32_t x) -> int64_t {
    int r = (int)ix.size();
    for (int p = 0; p < r; ++p)
      if (ix[p] == x) return int64_t(1) << (r - 1 - p);
    return 0;
  };
  std::vector<int64_t> sn(rr), st(rr), kn(ks), kt(ks);
  for (int j = 0; j < rr; ++j) {
    sn[j] = stride(n.ix, r.ix[j]);
    st[j] = stride(t.ix, r.ix[j]);
  }
  for (int j = 0; j < ks; ++j) {
    kn[j] = stride(n.ix, shared[j]);
    kt[j] = stride(t.ix, shared[j]);
  }
  for (int64_t o = 0; o < (int64_t(1) << rr); ++o) {
    int64_t bn = 0, bt = 0;
    for (int j = 0; j < rr; ++j)
      if ((o >> (rr - 1 - j)) & 1) {
        bn += sn[j];
        bt += st[j];
      }
    cd acc = 0;
    for (int64_t z = 0; z < (int64_t(1) << ks); ++z) {
      int64_t on = bn, ot = bt;
      for (int j = 0; j < ks; ++j)
        if ((z >> (ks - 1 - j)) & 1) {
          on += kn[j];
          ot += kt[j];
        }
      acc += n.d[on] * t.d[ot];
    }
    r.d[o] = acc;
  }
  (void)rn;
  (void)rt;
  return r;
}

}  // namespace

extern "C" ltn_status ltn_network_build(int32_t n_qubits, const ltn_gate* gates, int32_t n_gates,
                                        const int32_t* closed_bits, int32_t absorb,
                                        ltn_netbuf** out) {
  return ltn::guarded([&] {
    using ltn::require;
    require(out != nullptr, "out is NULL");
    require(n_qubits >= 1 && n_qubits <= 1024, "bad qubit count");
    require(n_gates >= 0 && (n_gates == 0 || gates), "bad gate list");
    require(closed_bits != nullptr, "closed_bits is NULL");
    std::vector<int32_t> wire(n_qubits);
    std::map<int32_t, T> tens;  // id -> tensor (ordered by id)
    int32_t tid = 0, next_index = n_qubits;
    for (int32_t q = 0; q < n_qubits; ++q) {
      wire[q] = q;
      tens[tid++] = T{{q}, {1.0, 0.0}, -1};
    }
    for (int32_t i = 0; i < n_gates; ++i) {
      const ltn_gate& g = gates[i];
      bool two = g.q1 >= 0;
      require(g.q0 >= 0 && g.q0 < n_qubits && (!two || (g.q1 < n_qubits && g.q1 != g.q0)),
              "gate " + std::to_string(i) + " has bad qubits");
      require(g.kind != LTN_GATE_FSIM || two, "fsim needs two qubits");
      require(!(g.kind >= LTN_GATE_SQRT_X && g.kind <= LTN_GATE_SQRT_W) || !two,
              "single-qubit gate given two qubits");
      require(g.kind != LTN_GATE_U3 || (!two && g.param_id >= 0), "u3 needs one qubit and a param_id");
      T t;
      t.d = gate_matrix(g);
      if (two) {
        int32_t o0 = next_index++, o1 = next_index++;
        t.ix = {o0, o1, wire[g.q0], wire[g.q1]};
        wire[g.q0] = o0;
        wire[g.q1] = o1;
      } else {
        int32_t o = next_index++;
        t.ix = {o, wire[g.q0]};
        wire[g.q0] = o;
      }
      t.param = g.kind == LTN_GATE_U3 ? g.param_id : -1;
      tens[tid++] = t;
    }
    std::vector<int32_t> open_ids;
    for (int32_t q = 0; q < n_qubits; ++q) {
      int32_t b = closed_bits[q];
      require(b >= -1 && b <= 1, "closed_bits entries must be -1, 0 or 1");
      if (b < 0) {
        open_ids.push_back(wire[q]);
        continue;
      }
      T t{{wire[q]}, {b == 0 ? 1.0 : 0.0, b == 1 ? 1.0 : 0.0}, -1};
      tens[tid++] = t;
    }
    // absorption: lowest-id tensor of rank <= 2 that is not a u3 leaf and has
    // a non-u3 neighbour goes into its lowest-id such neighbour
    if (absorb) {
      std::map<int32_t, std::vector<int32_t>> owners;  // index -> tensor ids
      for (auto& kv : tens)
        for (int32_t x : kv.second.ix) owners[x].push_back(kv.first);
      for (;;) {
        int32_t pick = -1, into = -1;
        for (auto& kv : tens) {
          const T& t = kv.second;
          if (t.param >= 0 || t.ix.size() > 2) continue;
          int32_t best = -1;
          if (t.ix.empty()) {
            for (auto& kv2 : tens)
              if (kv2.first != kv.first && kv2.second.param < 0) {
                best = kv2.first;
                break;
              }
          } else {
            for (int32_t x : t.ix)
              for (int32_t u : owners[x])
                if (u != kv.first && tens[u].param < 0 && (best < 0 || u < best)) best = u;
          }
          if (best >= 0) {
            pick = kv.first;
            into = best;
            break;
          }
        }
        if (pick < 0) break;
        T merged = merge(tens[into], tens[pick]);
        for (int32_t x : tens[pick].ix) {
          auto& o = owners[x];
          o.erase(std::remove(o.begin(), o.end(), pick), o.end());
        }
        for (int32_t x : tens[into].ix) {
          auto& o = owners[x];
          o.erase(std::remove(o.begin(), o.end(), into), o.end());
        }
        for (int32_t x : merged.ix) owners[x].push_back(into);
        tens[into] = std::move(merged);
        tens.erase(pick);
      }
    }
    // renumber indices densely in ascending old id
    std::map<int32_t, int32_t> remap;
    for (auto& kv : tens)
      for (int32_t x : kv.second.ix) remap[x] = 0;
    int32_t k = 0;
    for (auto& kv : remap) kv.second = k++;
    auto nb = new ltn_netbuf();
    nb->n_indices = k;
    nb->leaf_off.push_back(0);
    for (auto& kv : tens) {
      const T& t = kv.second;
      for (int32_t x : t.ix) nb->index_ids.push_back(remap[x]);
      nb->leaf_off.push_back((int64_t)nb->index_ids.size());
      for (const cd& v : t.d) {
        nb->data128.push_back(v.real());
        nb->data128.push_back(v.imag());
        nb->data64.push_back((float)v.real());
        nb->data64.push_back((float)v.imag());
      }
      nb->param.push_back(t.param);
    }
    for (int32_t x : open_ids) nb->open_ids.push_back(remap.count(x) ? remap[x] : -1);
    for (int32_t x : nb->open_ids)
      if (x < 0) {
        delete nb;
        ltn::fail(LTN_E_INVALID, "an open wire vanished during absorption");
      }
    *out = nb;
  });
}

extern "C" ltn_status ltn_netbuf_view(const ltn_netbuf* nb, ltn_network* v) {
  return ltn::guarded([&] {
    ltn::require(nb && v, "NULL argument");
    v->n_leaves = (int32_t)nb->param.size();
    v->leaf_off = nb->leaf_off.data();
    v->index_ids = nb->index_ids.data();
    v->leaf_data = nb->data64.data();
    v->n_open = (int32_t)nb->open_ids.size();
    v->open_ids = nb->open_ids.data();
    v->n_indices = nb->n_indices;
    v->param_leaf = nb->param.data();
  });
}

extern "C" ltn_status ltn_netbuf_data128(const ltn_netbuf* nb, const double** data) {
  return ltn::guarded([&] {
    ltn::require(nb && data, "NULL argument");
    *data = nb->data128.data();
  });
}

extern "C" void ltn_netbuf_free(ltn_netbuf* nb) { delete nb; }
