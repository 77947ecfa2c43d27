// Bit permutation of a batch of complex64 tensors:
//     out[b][y] = in[b][x],  bit perm[j] of y = bit j of x.
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

__device__ __forceinline__ uint64_t spread(uint64_t v, const int8_t* pos, int n) {
  uint64_t r = 0;
  for (int k = 0; k < n; ++k) r |= ((v >> k) & 1) << pos[k];
  return r;
}

// Bit maps are linear in the bits, so each tile-local map is the OR of a
// table over the low 6 tile bits and one over the high 6.
__global__ __launch_bounds__(256) void k_permute(const float2* __restrict__ in, float2* __restrict__ out,
                                                 PermuteDesc d) {
  __shared__ float2 tile[1 << kTileBits];
  __shared__ uint64_t src_lo[64], src_hi[64], dst_lo[64], dst_hi[64];
  __shared__ uint16_t map_lo[64], map_hi[64];
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
  __syncthreads();
  const int64_t per = int64_t(1) << d.rank;
  const int64_t outer = int64_t(1) << d.n_outer;
  const int nt = 1 << d.n_tile;
  const int lomask = (1 << nlo) - 1;
  for (int64_t blk = blockIdx.x; blk < outer * d.batch; blk += gridDim.x) {
    const int64_t b = blk / outer, o = blk % outer;
    const uint64_t sbase = spread((uint64_t)o, d.outer_src, d.n_outer);
    const uint64_t dbase = spread((uint64_t)o, d.outer_dst, d.n_outer);
    const float2* src = in + b * per;
    float2* dst = out + b * per;
    // read in source order (tile bit k = source bit tile_src[k], ascending)
    for (int l = threadIdx.x; l < nt; l += blockDim.x)
      tile[l] = src[sbase | src_lo[l & lomask] | src_hi[l >> nlo]];
    __syncthreads();
    // write in destination order
    for (int q = threadIdx.x; q < nt; q += blockDim.x)
      dst[dbase | dst_lo[q & lomask] | dst_hi[q >> nlo]] = tile[map_lo[q & lomask] | map_hi[q >> nlo]];
    __syncthreads();
  }
}

}  // namespace

void launch_permute(const float2* in, float2* out, const PermuteDesc& d, hipStream_t st) {
  int64_t blocks = (int64_t(1) << d.n_outer) * d.batch;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_permute, dim3((unsigned)blocks), dim3(256), 0, st, in, out, d);
}

}  // namespace ltn
