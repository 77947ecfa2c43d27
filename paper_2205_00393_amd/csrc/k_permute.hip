// Bit permutation of a batch of complex64 tensors:
//     out[b][y] = in[b][x],  bit perm[j] of y = bit j of x
// (optionally conjugated on the way: the sign bit of the imaginary part is
// flipped).
// Each block moves one tile: the source bits T = the lowest 5 source bits
// plus the source bits that land on the lowest 5 destination bits, filled
// up with the next source bits to 12; the other bits are fixed per block. The tile is read in source order
// into LDS and written in destination order, so both HBM sides move runs of
// 2^t consecutive elements. Runs of bits that keep their neighbours need no
// special casing: they are simply part of the runs.
#include "kernels.h"

namespace ltn {

namespace {

constexpr int kTileBits = 12;  // up to 4096 elements (32 KiB) per tile

// bit k of v goes to bit pos[k]
__device__ __forceinline__ uint64_t spread(uint64_t v, const int8_t* pos, int n) {
  uint64_t r = 0;
  for (int k = 0; k < n; ++k) r |= ((v >> k) & 1) << pos[k];
  return r;
}

// Bit maps are linear in the bits, so each tile-local map is the OR of a
// table over the low 6 tile bits and one over the high 6. Source bit 0 and
// destination bit 0 are always tile bits (the lowest of each order), so
// tile elements 2 j and 2 j + 1 are neighbours in HBM on both sides: every
// thread moves pairs j = tid + 256 i (i < 8) with one 16-byte load and one
// 16-byte store; their offsets are fixed per thread and computed once, and a
// block's 8 loads are issued back to back.
// LDS slot of tile element l: l with its low 5 bits XORed by swz_tab[l >> 5],
// chosen on the host so that the 32 elements one half-wave reads in
// destination order fall into 32 distinct bank pairs.
constexpr int kThreads = 256, kPer = (1 << kTileBits) / kThreads, kPairs = kPer / 2;
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// Elements are moved as 64-bit words (pure data movement, bit-exact); the
// conjugating variant flips the sign bit of each imaginary part.
template <bool CONJ>
__global__ __launch_bounds__(kThreads) void k_permute(const uint64_t* __restrict__ in,
                                                      uint64_t* __restrict__ out, PermuteDesc d) {
  __shared__ uint64_t tile[1 << kTileBits];
  __shared__ uint64_t src_lo[64], src_hi[64], dst_lo[64], dst_hi[64];
  __shared__ uint16_t map_lo[64], map_hi[64];
  __shared__ uint8_t swz_tab[1 << (kTileBits - 5)];
  const int nlo = d.n_tile < 6 ? d.n_tile : 6, nhi = d.n_tile - nlo;
  for (int e = threadIdx.x; e < 64; e += blockDim.x) {
    src_lo[e] = spread((uint64_t)e, d.tile_src, nlo);
    src_hi[e] = spread((uint64_t)e, d.tile_src + nlo, nhi);
    dst_lo[e] = spread((uint64_t)e, d.tile_dst, nlo);
    dst_hi[e] = spread((uint64_t)e, d.tile_dst + nlo, nhi);
    uint64_t ml = 0, mh = 0;
    for (int r = 0; r < nlo; ++r) ml |= ((uint64_t)(e >> r) & 1) << d.dst_tile[r];
    for (int r = 0; r < nhi; ++r) mh |= ((uint64_t)(e >> r) & 1) << d.dst_tile[nlo + r];
    map_lo[e] = (uint16_t)ml;
    map_hi[e] = (uint16_t)mh;
  }
  for (int h = threadIdx.x; h < (1 << (kTileBits - 5)); h += blockDim.x) {
    int m = 0;
    for (int k = 0; k < kTileBits - 5; ++k)
      if ((h >> k) & 1) m ^= d.swz[k];
    swz_tab[h] = (uint8_t)m;
  }
  __syncthreads();
  const int nt = 1 << d.n_tile;
  const int lomask = (1 << nlo) - 1;
  const int tid = threadIdx.x;
  const int64_t per = int64_t(1) << d.rank;
  const int64_t outer = int64_t(1) << d.n_outer;
  const uint64_t flip = CONJ ? (1ull << 63) : 0ull;
  if (nt < 2) {
    // rank-0 tensors: one element per batch entry
    for (int64_t blk = blockIdx.x * (int64_t)kThreads + tid; blk < d.batch; blk += (int64_t)gridDim.x * kThreads)
      out[blk] = in[blk] ^ flip;
    return;
  }
  uint64_t soff[kPairs], doff[kPairs];
  int ws0[kPairs], ws1[kPairs], rs0[kPairs], rs1[kPairs];
  auto rslot = [&](int l) {
    const int t = map_lo[l & lomask] | map_hi[l >> nlo];
    return t ^ swz_tab[t >> 5];
  };
#pragma unroll
  for (int i = 0; i < kPairs; ++i) {
    const int l = 2 * (tid + kThreads * i);
    if (l < nt) {
      soff[i] = src_lo[l & lomask] | src_hi[l >> nlo];
      doff[i] = dst_lo[l & lomask] | dst_hi[l >> nlo];
      ws0[i] = l ^ swz_tab[l >> 5];
      ws1[i] = (l + 1) ^ swz_tab[(l + 1) >> 5];
      rs0[i] = rslot(l);
      rs1[i] = rslot(l + 1);
    }
  }
  // Blocks are persistent (a few per CU, so that the tables above are built
  // once per block): the next tile's loads are issued as soon as the current
  // tile sits in LDS, and overlap its LDS reads and HBM writes.
  const int64_t tiles = outer * d.batch;
  auto fetch = [&](int64_t blk, u64x2* w) {
    const int64_t b = blk / outer, o = blk % outer;
    const uint64_t* src = in + b * per + spread((uint64_t)o, d.outer_src, d.n_outer);
#pragma unroll
    for (int i = 0; i < kPairs; ++i)
      if (2 * (tid + kThreads * i) < nt)
        w[i] = __builtin_nontemporal_load(reinterpret_cast<const u64x2*>(src + soff[i]));
  };
  u64x2 nx[kPairs];
  if (blockIdx.x < tiles) fetch(blockIdx.x, nx);
  for (int64_t blk = blockIdx.x; blk < tiles; blk += gridDim.x) {
    const int64_t b = blk / outer, o = blk % outer;
    uint64_t* dst = out + b * per + spread((uint64_t)o, d.outer_dst, d.n_outer);
    u64x2 v[kPairs];
#pragma unroll
    for (int i = 0; i < kPairs; ++i)
      if (2 * (tid + kThreads * i) < nt) {
        tile[ws0[i]] = nx[i].x;
        tile[ws1[i]] = nx[i].y;
      }
    __syncthreads();
    if (blk + gridDim.x < tiles) fetch(blk + gridDim.x, nx);
#pragma unroll
    for (int i = 0; i < kPairs; ++i)
      if (2 * (tid + kThreads * i) < nt) {
        v[i].x = tile[rs0[i]] ^ flip;
        v[i].y = tile[rs1[i]] ^ flip;
      }
#pragma unroll
    for (int i = 0; i < kPairs; ++i)
      if (2 * (tid + kThreads * i) < nt)
        __builtin_nontemporal_store(v[i], reinterpret_cast<u64x2*>(dst + doff[i]));
    __syncthreads();
  }
}

}  // namespace

void launch_permute(const float2* in, float2* out, const PermuteDesc& d, hipStream_t st) {
  // persistent blocks: 3 per CU on 256 CUs (registers allow 3 waves per SIMD)
  int64_t blocks = (int64_t(1) << d.n_outer) * d.batch;
  if (blocks > 768) blocks = 768;
  if (d.flip)
    hipLaunchKernelGGL(k_permute<true>, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                       reinterpret_cast<const uint64_t*>(in), reinterpret_cast<uint64_t*>(out), d);
  else
    hipLaunchKernelGGL(k_permute<false>, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                       reinterpret_cast<const uint64_t*>(in), reinterpret_cast<uint64_t*>(out), d);
}

}  // namespace ltn
