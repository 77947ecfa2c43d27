// Contraction steps with few outputs and a long sum: m, n <= 3 (at most 64
// outputs per slice) and up to 2^40 summed elements, as in the last steps
// of a tree, where two large tensors meet and only the open indices stay.
// Such a step reads 8 (2^(m+k) + 2^(n+k)) bytes and is bound by HBM, but
// one output per thread (or per 64 lanes) leaves the chip nearly idle. The
// sum is split instead: block (chunk, slice) reduces 2^kc consecutive k
// for every output (coalesced reads of all 2^m rows of A and 2^n rows of B,
// FP32 accumulators in registers, then a wave and block reduction), writes
// one FP32 partial per output; a second kernel adds the partials of each
// output in FP32 in a fixed order (strided per thread, then a pairwise tree
// over the block), so the result does not depend on timing.
#include "kernels.h"

namespace ltn {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint64_t pdep_s(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  for (uint64_t bit = 1; mask; bit <<= 1) {
    const uint64_t low = mask & (~mask + 1);
    if (x & bit) r |= low;
    mask ^= low;
  }
  return r;
}

template <int M, int N>
__global__ __launch_bounds__(kThreads) void k_skinny_partial(SkinnyDesc d, int kc_bits) {
  const int64_t chunk = blockIdx.x, chunks = gridDim.x;
  const int b = blockIdx.y;
  const int64_t K = int64_t(1) << d.k, KC = int64_t(1) << kc_bits;
  const float2* A = d.A + b * d.sA + chunk * KC;
  const float2* B = d.B + b * d.sB + chunk * KC;
  float2 acc[M][N];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) acc[i][j] = make_float2(0.f, 0.f);
  for (int64_t kk = threadIdx.x; kk < KC; kk += kThreads) {
    float2 a[M], bv[N];
#pragma unroll
    for (int i = 0; i < M; ++i) a[i] = A[i * K + kk];
#pragma unroll
    for (int j = 0; j < N; ++j) bv[j] = B[j * K + kk];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        acc[i][j].x += a[i].x * bv[j].x - a[i].y * bv[j].y;
        acc[i][j].y += a[i].x * bv[j].y + a[i].y * bv[j].x;
      }
  }
  __shared__ float2 red[kThreads / 64][M * N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      float x = acc[i][j].x, y = acc[i][j].y;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off, 64);
        y += __shfl_xor(y, off, 64);
      }
      if (lane == 0) red[wave][i * N + j] = make_float2(x, y);
    }
  __syncthreads();
  for (int e = threadIdx.x; e < M * N; e += kThreads) {
    float2 s = red[0][e];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) {
      s.x += red[w][e].x;
      s.y += red[w][e].y;
    }
    d.part[(b * chunks + chunk) * (M * N) + e] = s;
  }
}

// One block per (output, slice): the chunk partials are added in FP32 in a
// fixed order (at most 16 per thread, strided, then a pairwise tree over
// the block).
__global__ __launch_bounds__(kThreads) void k_skinny_reduce(SkinnyDesc d, int64_t chunks) {
  const int e = blockIdx.x, b = blockIdx.y;
  const int mn = 1 << (d.m + d.n);
  float x = 0.f, y = 0.f;
  for (int64_t c = threadIdx.x; c < chunks; c += kThreads) {
    const float2 v = d.part[(b * chunks + c) * mn + e];
    x += v.x;
    y += v.y;
  }
  __shared__ float rx[kThreads], ry[kThreads];
  rx[threadIdx.x] = x;
  ry[threadIdx.x] = y;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      rx[threadIdx.x] += rx[threadIdx.x + h];
      ry[threadIdx.x] += ry[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint64_t full = (1ull << (d.m + d.n)) - 1;
    const uint64_t i = (uint64_t)e >> d.n, j = (uint64_t)e & ((1ull << d.n) - 1);
    const uint64_t addr = pdep_s(i, d.cmask) | pdep_s(j, ~d.cmask & full);
    const float2 out = make_float2(rx[0], ry[0]);
    d.C[b * d.sC + addr] = out;
    if (d.scale_c) raise_max(d.scale_c + b, fmaxf(fabsf(out.x), fabsf(out.y)));
  }
}

template <int M>
void launch_m(const SkinnyDesc& d, dim3 grid, int kc, hipStream_t st) {
  switch (d.n) {
    case 0: hipLaunchKernelGGL((k_skinny_partial<M, 1>), grid, dim3(kThreads), 0, st, d, kc); break;
    case 1: hipLaunchKernelGGL((k_skinny_partial<M, 2>), grid, dim3(kThreads), 0, st, d, kc); break;
    case 2: hipLaunchKernelGGL((k_skinny_partial<M, 4>), grid, dim3(kThreads), 0, st, d, kc); break;
    default: hipLaunchKernelGGL((k_skinny_partial<M, 8>), grid, dim3(kThreads), 0, st, d, kc); break;
  }
}

}  // namespace

bool skinny_fits(int m, int k, int n) { return m >= 0 && m <= 3 && n >= 0 && n <= 3 && k >= 0 && k <= 40; }

// chunks of 2^11 elements (8 per thread), at most 2^12 chunks
int skinny_chunk_bits(int k) {
  int kc = k < 11 ? k : 11;
  if (k - kc > 12) kc = k - 12;
  return kc;
}

int64_t skinny_part_elems(int m, int k, int n) {
  return (int64_t(1) << (k - skinny_chunk_bits(k))) << (m + n);
}

void launch_skinny(const SkinnyDesc& d, hipStream_t st) {
  const int kc = skinny_chunk_bits(d.k);
  const int64_t chunks = int64_t(1) << (d.k - kc);
  const dim3 grid((unsigned)chunks, (unsigned)d.nb);
  switch (d.m) {
    case 0: launch_m<1>(d, grid, kc, st); break;
    case 1: launch_m<2>(d, grid, kc, st); break;
    case 2: launch_m<4>(d, grid, kc, st); break;
    default: launch_m<8>(d, grid, kc, st); break;
  }
  hipLaunchKernelGGL(k_skinny_reduce, dim3(1u << (d.m + d.n), (unsigned)d.nb), dim3(kThreads), 0, st, d,
                     chunks);
}

}  // namespace ltn
