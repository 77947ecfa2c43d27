// Small kernels: slice-id fill, leaf gather, FP64 slice sum with placement,
// root cotangent gather, u3 leaves and their adjoint, zero fill, and the
// generic bit-addressed contraction used for the adjoint sweep and for
// steps too small for the MFMA GEMM.
#include "kernels.h"

namespace ltn {

namespace {

struct IdBlock {
  uint64_t v[64];
};

__global__ void k_set_ids(uint64_t* d, IdBlock blk, int n) {
  int i = threadIdx.x;
  if (i < n) d[i] = blk.v[i];
}

__global__ void k_set_range(uint64_t* d, uint64_t base, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = base + (uint64_t)i;
}

// wave-wide max, then one atomic per wave (non-negative floats order like
// their bit patterns)
__device__ __forceinline__ void record_max(uint32_t* slot, float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) raise_max(slot, v);
}

// one block per (chunk of kGatherChunk elements of a leaf, slice): chunks
// are numbered leaf after leaf (desc[l].chunk0 = first chunk of leaf l);
// when every leaf is one chunk, block x is leaf x, else a binary search
// over chunk0 finds the leaf
__global__ void k_gather(const GatherDesc* __restrict__ desc, int n_leaves, int64_t n_chunks,
                         const float2* __restrict__ src, float2* __restrict__ arena,
                         const uint64_t* __restrict__ ids, int nb, uint32_t* scales, int bstride) {
  const int64_t chunk = blockIdx.x;
  int leaf = (int)chunk;
  if (n_chunks != n_leaves) {
    int lo = 0, hi = n_leaves - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (desc[mid].chunk0 <= chunk)
        lo = mid;
      else
        hi = mid - 1;
    }
    leaf = lo;
  }
  const GatherDesc& g = desc[leaf];
  int b = blockIdx.y;
  uint64_t s = ids[b];
  int64_t base = g.src_off;
  for (int i = 0; i < g.nsl; ++i) base += (int64_t)((s >> g.sl_bit[i]) & 1) << g.sl_src_bit[i];
  int64_t n = int64_t(1) << g.rank;
  float2* dst = arena + g.dst_off + (int64_t)b * n;
  const int64_t c0 = (chunk - g.chunk0) * kGatherChunk;
  const int64_t c1 = c0 + kGatherChunk < n ? c0 + kGatherChunk : n;
  float vmax = 0.f;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    int64_t o = base;
    for (int j = 0; j < g.rank; ++j) o += ((c >> j) & 1) << g.src_bit[j];
    float2 v = src[o];
    vmax = fmaxf(vmax, fmaxf(fabsf(v.x), fabsf(v.y)));
    dst[c] = v;
  }
  if (scales) record_max(scales + g.tensor * (int64_t)bstride + b, vmax);
}

__device__ __forceinline__ uint64_t pdep(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  while (mask) {
    uint64_t low = mask & (~mask + 1);
    if (x & 1) r |= low;
    x >>= 1;
    mask &= mask - 1;
  }
  return r;
}

__device__ __forceinline__ uint64_t pext(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  int j = 0;
  while (mask) {
    uint64_t low = mask & (~mask + 1);
    if (x & low) r |= 1ull << j;
    ++j;
    mask &= mask - 1;
  }
  return r;
}

struct SliceOut {
  int32_t sl[32];
  int32_t ob[32];
};

__device__ __forceinline__ uint64_t placement(uint64_t e, uint64_t out_mask, const SliceOut& so,
                                              int n_sl, uint64_t s) {
  uint64_t p = pdep(e, out_mask);
  for (int i = 0; i < n_sl; ++i) p |= ((s >> so.sl[i]) & 1) << so.ob[i];
  return p;
}

// out[place(s_b, e)] += root[b][e] in FP64. Two forms, both in a fixed
// order (reruns are bit-identical) and without atomics: every target an
// element e can reach has e's unsliced open bits, so the work of one e
// never meets another's.
//
// Large roots: one thread per root element, b in ascending order (reads
// coalesced along e).
__global__ void k_reduce(const float2* __restrict__ root, int rank, uint64_t out_mask, SliceOut so,
                         int n_sl, const uint64_t* __restrict__ ids, int nb, double* out) {
  int64_t n = int64_t(1) << rank;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (n_sl == 0) {
      double re = 0, im = 0;
      for (int b = 0; b < nb; ++b) {
        float2 v = root[(int64_t)b * n + e];
        re += (double)v.x;
        im += (double)v.y;
      }
      uint64_t p = pdep((uint64_t)e, out_mask);
      out[2 * p] += re;
      out[2 * p + 1] += im;
    } else {
      for (int b = 0; b < nb; ++b) {
        float2 v = root[(int64_t)b * n + e];
        uint64_t p = placement((uint64_t)e, out_mask, so, n_sl, ids[b]);
        out[2 * p] += (double)v.x;
        out[2 * p + 1] += (double)v.y;
      }
    }
  }
}

// Small roots and many slices: one wave per root element, the batch
// across its lanes 64 slices at a time. Without sliced open indices every
// slice adds into the same target: a fixed butterfly of FP64 shuffles sums
// each chunk, lane 0 adds the chunks in order and writes once. With sliced
// open indices a slice's target also carries its sliced open bits (its
// key): the wave sorts (key, lane) pairs with a bitonic network of
// shuffles, fetches the values in that order, and a segmented FP64 shuffle
// scan over the sorted lanes leaves each key's sum on the last lane of its
// run, which writes it. The addition tree depends only on the keys' lane
// positions, so reruns are bit-identical. Up to four chunks are loaded
// before the first is summed; chunks are separated by a barrier, so a chunk
// sees the writes of the chunks before it.
__global__ void __launch_bounds__(64) k_reduce_lanes(const float2* __restrict__ root, int rank,
                                                     uint64_t out_mask, SliceOut so, int n_sl,
                                                     const uint64_t* __restrict__ ids, int nb,
                                                     double* out) {
  const int lane = threadIdx.x;
  const int64_t n = int64_t(1) << rank;
  for (int64_t e = blockIdx.x; e < n; e += gridDim.x) {
    const uint64_t base = pdep((uint64_t)e, out_mask);
    if (n_sl == 0) {
      double re = 0, im = 0;
      for (int c = 0; c < nb; c += 64) {
        const int b = c + lane;
        double xr = 0, xi = 0;
        if (b < nb) {
          const float2 v = root[(int64_t)b * n + e];
          xr = v.x;
          xi = v.y;
        }
        for (int off = 1; off < 64; off <<= 1) {
          xr += __shfl_xor(xr, off);
          xi += __shfl_xor(xi, off);
        }
        re += xr;
        im += xi;
      }
      if (lane == 0) {
        out[2 * base] += re;
        out[2 * base + 1] += im;
      }
    } else {
      for (int c0 = 0; c0 < nb; c0 += 256) {
        float2 v[4];
        uint64_t id[4], key[4];
        uint32_t ck[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {  // all loads issued before any use
          const int b = c0 + 64 * j + lane;
          v[j] = make_float2(0.f, 0.f);
          id[j] = 0;
          if (b < nb) {
            v[j] = root[(int64_t)b * n + e];
            id[j] = ids[b];
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          key[j] = 0;
          ck[j] = 0;
          if (c0 + 64 * j < nb)
            for (int i = 0; i < n_sl; ++i) {
              const uint64_t bit = (id[j] >> so.sl[i]) & 1;
              key[j] |= bit << so.ob[i];
              ck[j] |= (uint32_t)bit << i;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = c0 + 64 * j;
          if (c >= nb) break;
          // sort key: compact key above the lane (lanes past the batch last)
          const uint64_t grp = c + lane < nb ? (uint64_t)ck[j] : (1ull << 32);
          uint64_t sk = (grp << 6) | (uint64_t)lane;
          for (int k = 2; k <= 64; k <<= 1)
            for (int h = k >> 1; h > 0; h >>= 1) {
              const uint64_t o = __shfl_xor(sk, h, 64);
              const bool up = (lane & k) == 0, low = (lane & h) == 0;
              sk = (low == up) ? (o < sk ? o : sk) : (o > sk ? o : sk);
            }
          const int src = (int)(sk & 63);
          const uint64_t g = sk >> 6;
          double sr = (double)__shfl(v[j].x, src, 64);
          double si = (double)__shfl(v[j].y, src, 64);
          const uint64_t p = base | __shfl(key[j], src, 64);
          for (int d = 1; d < 64; d <<= 1) {
            const double pr = __shfl_up(sr, d, 64), pi = __shfl_up(si, d, 64);
            const uint64_t pg = __shfl_up(g, d, 64);
            if (lane >= d && pg == g) {
              sr += pr;
              si += pi;
            }
          }
          const uint64_t ng = __shfl_down(g, 1, 64);
          if (g < (1ull << 32) && (lane == 63 || ng != g)) {
            out[2 * p] += sr;
            out[2 * p + 1] += si;
          }
          __syncthreads();
        }
      }
    }
  }
}

__global__ void k_root_cot(const double* __restrict__ cot, int rank, uint64_t out_mask, SliceOut so,
                           int n_sl, const uint64_t* __restrict__ ids, int nb, float2* rootcot) {
  int64_t n = int64_t(1) << rank;
  int64_t total = n * nb;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t b = i >> rank, e = i & (n - 1);
    uint64_t p = placement((uint64_t)e, out_mask, so, n_sl, ids[b]);
    rootcot[i] = make_float2((float)cot[2 * p], (float)cot[2 * p + 1]);
  }
}

struct C2 {
  double re, im;
};
__device__ __forceinline__ C2 cmul(C2 a, C2 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ C2 cexpi(double t) { return {cos(t), sin(t)}; }

// U = Rz(a) Ry(b) Rz(c) and its three partial derivatives, [out][in]
__device__ void u3_parts(const double* ang, C2 U[4], C2 dU[3][4]) {
  double a = ang[0], b = ang[1], c = ang[2];
  C2 ea = cexpi(-0.5 * a), eac = {ea.re, -ea.im};
  C2 ec = cexpi(-0.5 * c), ecc = {ec.re, -ec.im};
  double cb = cos(0.5 * b), sb = sin(0.5 * b);
  C2 cbv = {cb, 0}, sbv = {sb, 0}, msb = {-sb, 0};
  U[0] = cmul(cmul(ea, cbv), ec);
  U[1] = cmul(cmul(ea, msb), ecc);
  U[2] = cmul(cmul(eac, sbv), ec);
  U[3] = cmul(cmul(eac, cbv), ecc);
  // d/da: rows scaled by -i/2 (row 0) and +i/2 (row 1)
  C2 mi2 = {0, -0.5}, pi2 = {0, 0.5};
  dU[0][0] = cmul(mi2, U[0]);
  dU[0][1] = cmul(mi2, U[1]);
  dU[0][2] = cmul(pi2, U[2]);
  dU[0][3] = cmul(pi2, U[3]);
  // d/db: Rz(a) dRy(b) Rz(c), dRy = 1/2 [[-s, -c], [c, -s]]
  C2 hs = {-0.5 * sb, 0}, hcm = {-0.5 * cb, 0}, hc = {0.5 * cb, 0};
  dU[1][0] = cmul(cmul(ea, hs), ec);
  dU[1][1] = cmul(cmul(ea, hcm), ecc);
  dU[1][2] = cmul(cmul(eac, hc), ec);
  dU[1][3] = cmul(cmul(eac, hs), ecc);
  // d/dc: columns scaled by -i/2 (col 0) and +i/2 (col 1)
  dU[2][0] = cmul(U[0], mi2);
  dU[2][1] = cmul(U[1], pi2);
  dU[2][2] = cmul(U[2], mi2);
  dU[2][3] = cmul(U[3], pi2);
}

__global__ void k_u3_build(const ParamLeaf* __restrict__ pl, int n, const double* __restrict__ ang,
                           float2* leafdata) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  C2 U[4], dU[3][4];
  u3_parts(ang + 3 * (int64_t)pl[i].gate, U, dU);
  for (int e = 0; e < 4; ++e) leafdata[pl[i].src_off + e] = make_float2((float)U[e].re, (float)U[e].im);
}

// leafgrad[4 i + o] += sum_b cot_b[canonical(o)] over the slices whose
// sliced values match the source element o (FP64, ascending b)
__global__ void k_leaf_cot(const ParamLeaf* __restrict__ pl, int n, const GatherDesc* __restrict__ gd,
                           const float2* __restrict__ arena, const uint64_t* __restrict__ ids, int nb,
                           double* leafgrad) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  int i = t >> 2, o = t & 3;
  const GatherDesc& g = gd[pl[i].gd];
  int64_t cnt = int64_t(1) << g.rank;
  double re = 0, im = 0;
  for (int b = 0; b < nb; ++b) {
    uint64_t s = ids[b];
    bool match = true;
    for (int q = 0; q < g.nsl; ++q)
      if ((((uint64_t)o >> g.sl_src_bit[q]) & 1) != ((s >> g.sl_bit[q]) & 1)) match = false;
    if (!match) continue;
    int64_t c = 0;
    for (int j = 0; j < g.rank; ++j) c |= (int64_t)((o >> g.src_bit[j]) & 1) << j;
    float2 v = arena[g.dst_off + (int64_t)b * cnt + c];
    re += (double)v.x;
    im += (double)v.y;
  }
  leafgrad[2 * t] += re;
  leafgrad[2 * t + 1] += im;
}

// dL/dtheta = Re sum conj(cot) dU/dtheta
__global__ void k_u3_adjoint(const ParamLeaf* __restrict__ pl, int n, const double* __restrict__ ang,
                             const double* __restrict__ lg, double* grad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  C2 U[4], dU[3][4];
  int g = pl[i].gate;
  u3_parts(ang + 3 * (int64_t)g, U, dU);
  for (int j = 0; j < 3; ++j) {
    double acc = 0;
    for (int e = 0; e < 4; ++e) {
      double cr = lg[8 * i + 2 * e], ci = lg[8 * i + 2 * e + 1];
      acc += cr * dU[j][e].re + ci * dU[j][e].im;
    }
    grad[3 * g + j] += acc;
  }
}

__global__ void k_fill_zero(uint4* p, size_t n16) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0, 0, 0, 0);
}

// masked increment: the next value of pdep(z, mask) after adding pdep(d, mask)
__device__ __forceinline__ uint64_t madd(uint64_t a, uint64_t d, uint64_t mask) {
  return ((a | ~mask) + d) & mask;
}

// blk / nblk: this block's index and the number of blocks working on d
template <int TK>
__device__ __forceinline__ void generic_body(const GenericDesc& d, uint64_t blk, uint64_t nblk) {
  const int per_block = 256 / TK;
  const int lane = threadIdx.x % TK;
  const uint64_t n_out = 1ull << (d.xb + d.yb);
  const uint64_t total = n_out * (uint64_t)d.nb;
  const uint64_t zc = 1ull << d.zb;
  const uint64_t zstep = pdep((uint64_t)TK, d.pz), zstepq = pdep((uint64_t)TK, d.qz);
  const uint64_t z0p = pdep((uint64_t)lane, d.pz), z0q = pdep((uint64_t)lane, d.qz);
  // running max of the outputs this lane wrote, per slice (flushed with an
  // atomic when the slice changes and once after the loop)
  uint64_t bcur = ~0ull;
  float vcur = 0.f;
  for (uint64_t g = blk * per_block + threadIdx.x / TK; g < total; g += nblk * per_block) {
    uint64_t b = g >> (d.xb + d.yb);
    uint64_t o = g & (n_out - 1);
    // o enumerates the output in linear order: recover x, y from its bits
    uint64_t omask = d.ox | d.oy;
    uint64_t oaddr = pdep(o, omask);
    uint64_t x = pext(oaddr, d.ox), y = pext(oaddr, d.oy);
    const float2* P = d.P + b * d.sP + pdep(x, d.px);
    const float2* Q = d.Q + b * d.sQ + pdep(y, d.qy);
    float re = 0.f, im = 0.f;
    uint64_t zp = z0p, zq = z0q;
    // four iterations at a time, their eight loads issued before any product
    // (a loop with one exit test per iteration keeps only two loads in flight)
    for (uint64_t z = lane; z < zc; z += 4 * TK) {
      float2 p[4], q[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool in = z + (uint64_t)j * TK < zc;
        p[j] = in ? P[zp] : make_float2(0.f, 0.f);
        q[j] = in ? Q[zq] : make_float2(0.f, 0.f);
        zp = madd(zp, zstep, d.pz);
        zq = madd(zq, zstepq, d.qz);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (d.conjQ) q[j].y = -q[j].y;
        re += p[j].x * q[j].x - p[j].y * q[j].y;
        im += p[j].x * q[j].y + p[j].y * q[j].x;
      }
    }
    if (TK > 1) {
#pragma unroll
      for (int off = TK / 2; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, TK);
        im += __shfl_xor(im, off, TK);
      }
    }
    if (lane == 0) {
      float2* O = d.out + b * d.sO + oaddr;
      if (d.accumulate) {
        float2 v = *O;
        *O = make_float2(v.x + re, v.y + im);
      } else {
        *O = make_float2(re, im);
      }
    }
    if (d.scale_out && lane == 0) {
      if (b != bcur) {
        if (bcur != ~0ull) raise_max(d.scale_out + bcur, vcur);
        bcur = b;
        vcur = 0.f;
      }
      vcur = fmaxf(vcur, fmaxf(fabsf(re), fabsf(im)));
    }
  }
  if (d.scale_out) {
    // every lane is active again here: one atomic per wave if all lanes that
    // hold a value share one slice, else one per lane
    uint64_t b0 = __shfl(bcur, 0, 64);
    bool same = __all(bcur == b0 || bcur == ~0ull);
    if (same && b0 != ~0ull) {
      float v = vcur;
      for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
      if ((threadIdx.x & 63) == 0) raise_max(d.scale_out + b0, v);
    } else if (!same && bcur != ~0ull && vcur > 0.f) {
      raise_max(d.scale_out + bcur, vcur);
    }
  }
}

template <int TK>
__global__ __launch_bounds__(256) void k_generic(GenericDesc d) {
  generic_body<TK>(d, blockIdx.x, gridDim.x);
}

// Several independent generic contractions in one launch: grid row y runs
// descriptor y (from device memory) for nb slices.
template <int TK>
__global__ __launch_bounds__(256) void k_generic_multi(const GenericDesc* descs, int nb) {
  GenericDesc d = descs[blockIdx.y];
  d.nb = nb;
  generic_body<TK>(d, blockIdx.x, gridDim.x);
}

int grid_for(uint64_t items, int per_block) {
  uint64_t blocks = (items + per_block - 1) / per_block;
  return (int)(blocks < 65536 ? (blocks ? blocks : 1) : 65536);
}

}  // namespace

void launch_set_ids(uint64_t* d_ids, const uint64_t* h_ids, int n, hipStream_t st) {
  for (int off = 0; off < n; off += 64) {
    IdBlock blk;
    int c = n - off < 64 ? n - off : 64;
    for (int i = 0; i < c; ++i) blk.v[i] = h_ids[off + i];
    hipLaunchKernelGGL(k_set_ids, dim3(1), dim3(64), 0, st, d_ids + off, blk, c);
  }
}

void launch_set_range(uint64_t* d_ids, uint64_t base, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_set_range, dim3((n + 255) / 256), dim3(256), 0, st, d_ids, base, n);
}

void launch_gather(const GatherDesc* d_desc, int n_leaves, int64_t n_chunks, int max_elems,
                   const float2* leafdata, float2* arena, const uint64_t* ids, int nb, uint32_t* scales,
                   int bstride, hipStream_t st) {
  int threads = max_elems >= 256 ? 256 : (max_elems >= 64 ? max_elems : 64);
  hipLaunchKernelGGL(k_gather, dim3((unsigned)n_chunks, nb), dim3(threads), 0, st, d_desc, n_leaves,
                     n_chunks, leafdata, arena, ids, nb, scales, bstride);
}

static SliceOut make_so(const int32_t* sl, const int32_t* ob, int n) {
  SliceOut so{};
  for (int i = 0; i < n && i < 32; ++i) {
    so.sl[i] = sl[i];
    so.ob[i] = ob[i];
  }
  return so;
}

void launch_reduce(const float2* root, int rank, uint64_t out_mask, const int32_t* sl_bits,
                   const int32_t* out_bits, int n_sl, const uint64_t* ids, int nb, double* out,
                   hipStream_t st) {
  uint64_t n = 1ull << rank;
  if (nb >= 4 && n <= 4096)
    hipLaunchKernelGGL(k_reduce_lanes, dim3((unsigned)n), dim3(64), 0, st, root, rank, out_mask,
                       make_so(sl_bits, out_bits, n_sl), n_sl, ids, nb, out);
  else
    hipLaunchKernelGGL(k_reduce, dim3(grid_for(n, 256)), dim3(256), 0, st, root, rank, out_mask,
                       make_so(sl_bits, out_bits, n_sl), n_sl, ids, nb, out);
}

void launch_root_cotangent(const double* cot, int rank, uint64_t out_mask, const int32_t* sl_bits,
                           const int32_t* out_bits, int n_sl, const uint64_t* ids, int nb,
                           float2* rootcot, hipStream_t st) {
  uint64_t n = (1ull << rank) * (uint64_t)nb;
  hipLaunchKernelGGL(k_root_cot, dim3(grid_for(n, 256)), dim3(256), 0, st, cot, rank, out_mask,
                     make_so(sl_bits, out_bits, n_sl), n_sl, ids, nb, rootcot);
}

void launch_u3_build(const ParamLeaf* d_pl, int n, const double* angles, float2* leafdata,
                     hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_u3_build, dim3((n + 63) / 64), dim3(64), 0, st, d_pl, n, angles, leafdata);
}

void launch_leaf_cot_accumulate(const ParamLeaf* d_pl, int n, const GatherDesc* gd,
                                const float2* cot_arena, const uint64_t* ids, int nb,
                                double* leafgrad, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_leaf_cot, dim3((4 * n + 127) / 128), dim3(128), 0, st, d_pl, n, gd,
                     cot_arena, ids, nb, leafgrad);
}

void launch_u3_adjoint(const ParamLeaf* d_pl, int n, const double* angles, const double* leafgrad,
                       double* angle_grad, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_u3_adjoint, dim3((n + 63) / 64), dim3(64), 0, st, d_pl, n, angles, leafgrad,
                     angle_grad);
}

void launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  size_t n16 = bytes / 16;
  if (n16 == 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n16, 256) < 4096 ? grid_for(n16, 256) : 4096),
                     dim3(256), 0, st, (uint4*)p, n16);
}

void launch_generic_multi(const GenericDesc* d_descs, int n, uint64_t max_outs, int nb, int tk,
                          hipStream_t st) {
  if (n <= 0) return;
  const uint64_t outs = max_outs * (uint64_t)nb;
  const int per_block = tk == 1 ? 256 : (tk == 8 ? 32 : 4);
  const dim3 grid((unsigned)grid_for(outs, per_block), (unsigned)n);
  switch (tk) {
    case 1: hipLaunchKernelGGL(k_generic_multi<1>, grid, dim3(256), 0, st, d_descs, nb); break;
    case 8: hipLaunchKernelGGL(k_generic_multi<8>, grid, dim3(256), 0, st, d_descs, nb); break;
    default: hipLaunchKernelGGL(k_generic_multi<64>, grid, dim3(256), 0, st, d_descs, nb); break;
  }
}

void launch_generic(const GenericDesc& d, int tk, hipStream_t st) {
  uint64_t outs = (1ull << (d.xb + d.yb)) * (uint64_t)d.nb;
  switch (tk) {
    case 1:
      hipLaunchKernelGGL(k_generic<1>, dim3(grid_for(outs, 256)), dim3(256), 0, st, d);
      break;
    case 8:
      hipLaunchKernelGGL(k_generic<8>, dim3(grid_for(outs, 32)), dim3(256), 0, st, d);
      break;
    default:
      hipLaunchKernelGGL(k_generic<64>, dim3(grid_for(outs, 4)), dim3(256), 0, st, d);
      break;
  }
}

}  // namespace ltn
