// Narrow contraction steps: C[merge(m, n)] = sum_k A[m][k] B[n][k] with
// small k and n (k + n <= 10, n <= 6) and many rows m, as in the stem steps that
// absorb a small tensor. Such a step is bound by HBM (it reads A once and
// writes C once, about (K N / (K + N)) / 2 complex MACs per 8 bytes), so
// the kernel is built around coalesced traffic:
//  * a tile of TM = 2^q consecutive rows of A is one contiguous chunk
//    (rows are 2^k contiguous elements); it is loaded with consecutive
//    lanes on consecutive addresses into LDS (row stride K + 1 elements, so
//    that lanes reading the same k of consecutive rows hit distinct banks);
//  * B (2^n x 2^k elements, <= 8 KiB) sits in LDS and is read by broadcast;
//  * each thread computes NCH outputs of one row, keeping the A element in
//    a register across them; results are staged in LDS in output-address
//    order and written out with consecutive lanes on consecutive addresses
//    where C's layout allows (tile output bits = the q lowest m positions
//    and all n positions of C).
// Tile-local maps are linear in the bits, so they are tables over 6-bit
// halves (built per block). Optional per-slice max recording of |re|, |im|
// for split-fp16 consumers, one atomic per wave.
#include "kernels.h"

namespace ltn {

namespace {

__device__ __forceinline__ uint64_t pdep_n(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  for (uint64_t bit = 1; mask; bit <<= 1) {
    uint64_t low = mask & (~mask + 1);
    if (x & bit) r |= low;
    mask ^= low;
  }
  return r;
}

// LDS: A tile (TM * KP elements, also the staging area of the TM * N
// outputs) then B (N * K elements); sized per launch.
// Each thread computes RPT rows (TM / RPT apart) x NCH columns of a tile:
// every A element read feeds NCH products, every B element RPT.
template <int NCH, int RPT>
__global__ __launch_bounds__(256) void k_narrow(NarrowDesc d) {
  extern __shared__ float2 lds[];
  float2* As = lds;
  float2* Bs = lds + d.a_elems;
  __shared__ uint64_t tT_lo[64], tT_hi[64];
  __shared__ uint16_t tR_lo[64], tR_hi[64], tN[64];
  const int tid = threadIdx.x;
  const int q = d.q, K = 1 << d.k, N = 1 << d.n, TM = 1 << q;
  const int KP = K == 1 ? 1 : K + 1;
  const int NC = N / NCH;
  const int HR = TM / RPT;  // rows per row group
  const int items = HR * NC;
  const int outs = TM * N;
  const int tile_elems = TM * K;
  for (int e = tid; e < 64; e += blockDim.x) {
    tT_lo[e] = pdep_n((uint64_t)e, d.tmask);
    tT_hi[e] = pdep_n((uint64_t)e << 6, d.tmask);
    tR_lo[e] = (uint16_t)pdep_n((uint64_t)e, d.rt);
    tR_hi[e] = (uint16_t)pdep_n((uint64_t)e << 6, d.rt);
    tN[e] = (uint16_t)pdep_n((uint64_t)e, d.nt);
  }
  __syncthreads();
  const int64_t tiles = int64_t(1) << (d.m - q);
  const int64_t work = tiles * d.nb;
  float vmax = 0.f;  // running maximum of |re|, |im| for the current slice
  for (int64_t it = blockIdx.x; it < work; it += gridDim.x) {
    const int64_t b = it / tiles, tile = it % tiles;
    const uint64_t m0 = (uint64_t)tile << q;
    const float2* Ab = d.A + b * d.sA + (int64_t)(m0 << d.k);
    const float2* Bb = d.B + b * d.sB;
    float2* Cb = d.C + b * d.sC + pdep_n(m0, d.cmask);
    for (int e = tid; e < N * K; e += 256) Bs[e] = Bb[e];
    if (K >= 2) {
      // two elements of one row per 16-byte load
      const float4* A4 = reinterpret_cast<const float4*>(Ab);
      for (int e2 = tid; e2 < tile_elems / 2; e2 += 256) {
        const float4 v = A4[e2];
        const int e = 2 * e2, at = (e >> d.k) * KP + (e & (K - 1));
        As[at] = make_float2(v.x, v.y);
        As[at + 1] = make_float2(v.z, v.w);
      }
    } else {
      for (int e = tid; e < tile_elems; e += 256) As[e] = Ab[e];
    }
    __syncthreads();
    constexpr int PER = 8 / (NCH * RPT);  // items per thread (<= 2048 outputs per tile)
    float2 acc[8];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int w = tid + 256 * i;
#pragma unroll
      for (int j = 0; j < NCH * RPT; ++j) acc[i * NCH * RPT + j] = make_float2(0.f, 0.f);
      if (w < items) {
        const int r0 = w & (HR - 1), nc = w / HR;
        const float2* arow = As + r0 * KP;
        const float2* bcol = Bs + nc * NCH * K;
        for (int kk = 0; kk < K; ++kk) {
          float2 a[RPT];
#pragma unroll
          for (int u = 0; u < RPT; ++u) a[u] = arow[u * HR * KP + kk];
#pragma unroll
          for (int j = 0; j < NCH; ++j) {
            const float2 bv = bcol[j * K + kk];
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
              float2& c = acc[(i * RPT + u) * NCH + j];
              c.x += a[u].x * bv.x - a[u].y * bv.y;
              c.y += a[u].x * bv.y + a[u].y * bv.x;
            }
          }
        }
      }
    }
    __syncthreads();  // A tile no longer read: stage the outputs over it
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int w = tid + 256 * i;
      if (w < items) {
        const int r0 = w & (HR - 1), nc = w / HR;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int r = r0 + u * HR;
          const int tr = tR_lo[r & 63] | tR_hi[r >> 6];
#pragma unroll
          for (int j = 0; j < NCH; ++j) {
            const float2 v = acc[(i * RPT + u) * NCH + j];
            As[tr | tN[nc * NCH + j]] = v;
            vmax = fmaxf(vmax, fmaxf(fabsf(v.x), fabsf(v.y)));
          }
        }
      }
    }
    __syncthreads();
    if ((d.tmask & 1) && outs >= 2) {
      // tile bit 0 is C's bit 0: outputs 2j and 2j + 1 are neighbours in C
      for (int t2 = tid; t2 < outs / 2; t2 += 256) {
        const int t = 2 * t2;
        const float2 v0 = As[t], v1 = As[t + 1];
        *reinterpret_cast<float4*>(Cb + (tT_lo[t & 63] | tT_hi[t >> 6])) = make_float4(v0.x, v0.y, v1.x, v1.y);
      }
    } else {
      for (int t = tid; t < outs; t += 256) Cb[tT_lo[t & 63] | tT_hi[t >> 6]] = As[t];
    }
    if (d.scale_c) {
      // flush the running maximum when the next tile of this block belongs
      // to another slice (or there is none)
      const int64_t nx = it + gridDim.x;
      if (nx >= work || nx / tiles != b) {
        float v = vmax;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
        if ((tid & 63) == 0) raise_max(d.scale_c + b, v);
        vmax = 0.f;
      }
    }
    __syncthreads();  // the next tile overwrites As and Bs
  }
}

__device__ __forceinline__ uint64_t madd_n(uint64_t a, uint64_t d, uint64_t mask) {
  return ((a | ~mask) + d) & mask;
}

// Rows form: one thread per row of A. A block takes 256 consecutive rows
// of one slice at a time; each thread issues the K / 2 16-byte loads of its
// row (contiguous) at once, multiplies by B (N x K, broadcast from LDS) and
// writes its N outputs. The output address of row r, column j is
// pdep(chunk, cmask) | pdep(thread, cmask) | pdep(j, ~cmask): the first
// part is advanced from chunk to chunk by a masked add, the second is fixed
// per thread, the third is a table.
template <int K, int N>
__global__ __launch_bounds__(256) void k_narrow_rows(NarrowDesc d) {
  __shared__ float2 Bs[N * K];
  __shared__ uint64_t pj[N];
  const int tid = threadIdx.x;
  const uint64_t full = (d.m + d.n) >= 64 ? ~0ull : ((1ull << (d.m + d.n)) - 1);
  if (tid < N) pj[tid] = pdep_n((uint64_t)tid, ~d.cmask & full);
  const uint64_t pt = pdep_n((uint64_t)tid, d.cmask);
  const int64_t R = int64_t(1) << d.m;
  const int64_t chunks = (R >> 8) * d.nb;
  const uint64_t step = pdep_n((uint64_t)gridDim.x << 8, d.cmask);
  int64_t b_loaded = -1, r_prev = -1;
  uint64_t base = 0;
  float vmax = 0.f;
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int64_t b = (c << 8) >> d.m;
    const int64_t r0 = (c << 8) - (b << d.m);
    const float2* Ar = d.A + b * d.sA + (r0 + tid) * K;
    float2 a[K];
    if constexpr (K >= 2) {
#pragma unroll
      for (int kp = 0; kp < K / 2; ++kp) {
        const float4 v = reinterpret_cast<const float4*>(Ar)[kp];
        a[2 * kp] = make_float2(v.x, v.y);
        a[2 * kp + 1] = make_float2(v.z, v.w);
      }
    } else {
      a[0] = Ar[0];
    }
    if (b != b_loaded) {
      if (b_loaded >= 0 && d.scale_c) {
        float v = vmax;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
        if ((tid & 63) == 0) raise_max(d.scale_c + b_loaded, v);
        vmax = 0.f;
      }
      __syncthreads();  // the previous slice's B is no longer read
      const float2* Bb = d.B + b * d.sB;
      for (int e = tid; e < N * K; e += 256) Bs[e] = Bb[e];
      __syncthreads();
      b_loaded = b;
      base = pdep_n((uint64_t)r0, d.cmask);
    } else {
      base = r0 > r_prev ? madd_n(base, step, d.cmask) : pdep_n((uint64_t)r0, d.cmask);
    }
    r_prev = r0;
    float2 acc[N];
#pragma unroll
    for (int j = 0; j < N; ++j) acc[j] = make_float2(0.f, 0.f);
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const float2 bv = Bs[j * K + kk];
        acc[j].x += a[kk].x * bv.x - a[kk].y * bv.y;
        acc[j].y += a[kk].x * bv.y + a[kk].y * bv.x;
      }
    float2* Cb = d.C + b * d.sC + (base | pt);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      Cb[pj[j]] = acc[j];
      vmax = fmaxf(vmax, fmaxf(fabsf(acc[j].x), fabsf(acc[j].y)));
    }
  }
  if (d.scale_c && b_loaded >= 0) {
    float v = vmax;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((tid & 63) == 0) raise_max(d.scale_c + b_loaded, v);
  }
}

template <int K>
void launch_rows_k(const NarrowDesc& d, dim3 grid, hipStream_t st) {
  switch (d.n) {
    case 0: hipLaunchKernelGGL((k_narrow_rows<K, 1>), grid, dim3(256), 0, st, d); break;
    case 1: hipLaunchKernelGGL((k_narrow_rows<K, 2>), grid, dim3(256), 0, st, d); break;
    case 2: hipLaunchKernelGGL((k_narrow_rows<K, 4>), grid, dim3(256), 0, st, d); break;
    case 3: hipLaunchKernelGGL((k_narrow_rows<K, 8>), grid, dim3(256), 0, st, d); break;
    default: hipLaunchKernelGGL((k_narrow_rows<K, 16>), grid, dim3(256), 0, st, d); break;
  }
}

}  // namespace

bool narrow_fits(int m, int k, int n) { return k + n <= 10 && n <= 6 && m >= 0 && m <= 40; }

bool narrow_rows_fits(int m, int k, int n) { return k >= 0 && k <= 4 && n >= 0 && n <= 4 && m >= 8 && m <= 40; }

void launch_narrow(const NarrowDesc& d0, hipStream_t st) {
  NarrowDesc d = d0;
  if (d.cfg == 1) {
    const int64_t chunks = ((int64_t(1) << d.m) >> 8) * d.nb;
    const dim3 grid((unsigned)(chunks < 8192 ? chunks : 8192));
    switch (d.k) {
      case 0: launch_rows_k<1>(d, grid, st); break;
      case 1: launch_rows_k<2>(d, grid, st); break;
      case 2: launch_rows_k<4>(d, grid, st); break;
      case 3: launch_rows_k<8>(d, grid, st); break;
      default: launch_rows_k<16>(d, grid, st); break;
    }
    return;
  }
  const int K = 1 << d.k, N = 1 << d.n;
  int mx = d.k > d.n ? d.k : d.n;
  d.q = d.m < 11 - mx ? d.m : 11 - mx;
  // tile output bits: the q lowest m positions and all n positions of C
  const uint64_t full = (d.m + d.n) >= 64 ? ~0ull : ((1ull << (d.m + d.n)) - 1);
  const uint64_t npos = ~d.cmask & full;
  uint64_t mlow = 0, mm = d.cmask;
  for (int j = 0; j < d.q; ++j) {
    uint64_t low = mm & (~mm + 1);
    mlow |= low;
    mm ^= low;
  }
  d.tmask = mlow | npos;
  // positions, in tile order, of the row bits and of the n bits
  uint64_t rt = 0, nt = 0;
  int pos = 0;
  for (int bit = 0; bit < 64; ++bit) {
    const uint64_t v = 1ull << bit;
    if (!(d.tmask & v)) continue;
    if (mlow & v) rt |= 1ull << pos;
    if (npos & v) nt |= 1ull << pos;
    ++pos;
  }
  d.rt = rt;
  d.nt = nt;
  const int64_t tiles = (int64_t(1) << (d.m - d.q)) * d.nb;
  const int blocks = (int)(tiles < 65536 ? tiles : 65536);
  const int TM = 1 << d.q, KP = K == 1 ? 1 : K + 1;
  d.a_elems = TM * KP > TM * N ? TM * KP : TM * N;
  const size_t lds = (size_t)(d.a_elems + N * K) * sizeof(float2);
  // 2 rows x 4 columns per thread when the tile has >= 8 columns and >= 2
  // rows (6 LDS reads per 8 products), else one row x up to 8 columns
  if (N >= 8 && TM >= 2) {
    hipLaunchKernelGGL((k_narrow<4, 2>), dim3(blocks), dim3(256), lds, st, d);
    return;
  }
  const int nch = N >= 8 ? 8 : N;
  switch (nch) {
    case 1:
      hipLaunchKernelGGL((k_narrow<1, 1>), dim3(blocks), dim3(256), lds, st, d);
      break;
    case 2:
      hipLaunchKernelGGL((k_narrow<2, 1>), dim3(blocks), dim3(256), lds, st, d);
      break;
    case 4:
      hipLaunchKernelGGL((k_narrow<4, 1>), dim3(blocks), dim3(256), lds, st, d);
      break;
    default:
      hipLaunchKernelGGL((k_narrow<8, 1>), dim3(blocks), dim3(256), lds, st, d);
      break;
  }
}

}  // namespace ltn
