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

}  // namespace

bool narrow_fits(int m, int k, int n) { return k + n <= 10 && n <= 6 && m >= 0 && m <= 40; }

void launch_narrow(const NarrowDesc& d0, hipStream_t st) {
  NarrowDesc d = d0;
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
