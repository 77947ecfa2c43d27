// Fused sub-path (secondary slicing, Sec. 5.2): a run of stem steps in which
// the chain tensor absorbs one small tensor per step runs as one kernel.
// The indices of the run's input T_0 that survive to its output T_L (Sigma)
// are untouched inside the run, so every assignment sigma of them is an
// independent piece: the piece reads the 2^a contiguous elements of T_0 at
// sigma << a (its lowest a bits are the ones contracted inside), applies
// the L contractions to working tensors W_j (at most 2^rmax elements) held
// in LDS, and writes W_L once. HBM sees one read of T_0 and one write of T_L
// instead of a read and a write per step.
//
// Each wave owns one piece at a time (its own two LDS buffers), so the
// stages need only wave-level synchronisation; the waves of a block take
// the pieces of one round (same slice, so the small tensors staged in LDS
// are shared) and meet at a block barrier only when the slice changes.
// The next round's input is loaded into registers while the current piece
// is computed. Stage j: W_j[pos(r, n)] = sum_k W_{j-1}[r 2^k + k]
// Y_j[n 2^k + k] with pos(r, n) = pdep(r, cmask_j) | pdep(n, ~cmask_j),
// linear in the bits of r and n and read from per-stage tables over 6-bit
// halves; each lane computes a register block of up to 4 x 4 outputs, k in
// a lane-rotated order against bank conflicts.
#include "kernels.h"

namespace ltn {

namespace {

__device__ __forceinline__ uint64_t pdep_f(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  for (uint64_t bit = 1; mask; bit <<= 1) {
    uint64_t low = mask & (~mask + 1);
    if (x & bit) r |= low;
    mask ^= low;
  }
  return r;
}

constexpr int kInPer = 2048 / 64;  // input elements per lane (2^a <= 2^11)

// One stage for a lane: register blocks of RB rows x NB columns of W_j, with
// K = 2^kbits given at compile time when KC > 0 (the loops unroll without
// guards); KC = 0 takes K at run time.
template <int KC, int RB, int NB>
__device__ __forceinline__ void stage_blocks(const float2* in, float2* out, const float2* yb, int kbits,
                                             int m, int n, int rbits, int nbits,
                                             const uint16_t* rowPj, const uint16_t* nPj, int lane) {
  const int K = KC > 0 ? KC : (1 << kbits);
  const int nrb = 1 << (m - rbits);
  const int blocks = nrb << (n - nbits);
  const int r1 = rowPj[1], r2 = rowPj[2], c1 = nPj[1], c2 = nPj[2];
  const int roff[4] = {0, r1, r2, r1 | r2}, coff[4] = {0, c1, c2, c1 | c2};
  for (int w = lane; w < blocks; w += 64) {
    const int r0 = (w & (nrb - 1)) << rbits, n0 = (w >> (m - rbits)) << nbits;
    float2 acc[RB][NB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int q = 0; q < NB; ++q) acc[i][q] = make_float2(0.f, 0.f);
    const float2* ar = in + r0 * K;
    const float2* yr = yb + n0 * K;
    auto step = [&](int kk0) {
      const int kk = (kk0 + lane) & (K - 1);
      float2 x[RB], y[NB];
#pragma unroll
      for (int i = 0; i < RB; ++i) x[i] = ar[i * K + kk];
#pragma unroll
      for (int q = 0; q < NB; ++q) y[q] = yr[q * K + kk];
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          acc[i][q].x += x[i].x * y[q].x - x[i].y * y[q].y;
          acc[i][q].y += x[i].x * y[q].y + x[i].y * y[q].x;
        }
    };
    if constexpr (KC > 0) {
#pragma unroll
      for (int kk0 = 0; kk0 < KC; ++kk0) step(kk0);
    } else {
      for (int kk0 = 0; kk0 < K; ++kk0) step(kk0);
    }
    // positions are linear in the bits: base of the block, then the offsets
    // of rows 1..3 and columns 1..3 (disjoint bits)
    const int base = rowPj[r0 & 63] | rowPj[64 + (r0 >> 6)] | nPj[n0 & 63];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int q = 0; q < NB; ++q) out[base | roff[i] | coff[q]] = acc[i][q];
  }
}

template <int RB, int NB>
__device__ __forceinline__ void stage_k(const float2* in, float2* out, const float2* yb, int kbits,
                                        int m, int n, int rbits, int nbits, const uint16_t* rowPj,
                                        const uint16_t* nPj, int lane) {
  switch (kbits) {
    case 1: stage_blocks<2, RB, NB>(in, out, yb, kbits, m, n, rbits, nbits, rowPj, nPj, lane); break;
    case 2: stage_blocks<4, RB, NB>(in, out, yb, kbits, m, n, rbits, nbits, rowPj, nPj, lane); break;
    case 3: stage_blocks<8, RB, NB>(in, out, yb, kbits, m, n, rbits, nbits, rowPj, nPj, lane); break;
    default: stage_blocks<0, RB, NB>(in, out, yb, kbits, m, n, rbits, nbits, rowPj, nPj, lane); break;
  }
}

template <int WPB>
__global__ __launch_bounds__(64 * WPB) void k_fused(FusedDesc d) {
  extern __shared__ float2 lds[];
  const int W = 1 << d.rmax;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  float2* buf0 = lds + wave * 2 * W;
  float2* buf1 = buf0 + W;
  float2* Ys = lds + WPB * 2 * W;
  // rowP / nP: position in W_j of row r / column n (pdep over 6-bit halves)
  __shared__ uint16_t rowP[kFusedMaxStages][128], nP[kFusedMaxStages][128];
  __shared__ uint64_t wT[128];
  for (int e = tid; e < 64 * d.nstages; e += 64 * WPB) {
    const int j = e >> 6, v = e & 63;
    const FusedStage& s = d.st[j];
    const uint64_t full = (1ull << (s.m + s.n)) - 1;
    const uint64_t cm = s.cmask, ncm = ~s.cmask & full;
    rowP[j][v] = (uint16_t)pdep_f((uint64_t)v, cm);
    rowP[j][64 + v] = (uint16_t)pdep_f((uint64_t)v << 6, cm);
    nP[j][v] = (uint16_t)pdep_f((uint64_t)v, ncm);
    nP[j][64 + v] = (uint16_t)pdep_f((uint64_t)v << 6, ncm);
  }
  for (int v = tid; v < 64; v += 64 * WPB) {
    wT[v] = pdep_f((uint64_t)v, d.w_out);
    wT[64 + v] = pdep_f((uint64_t)v << 6, d.w_out);
  }
  // rounds of WPB consecutive pieces (2^nsig >= WPB pieces per slice, so a
  // round never spans two slices); each block takes a contiguous range
  const int64_t rounds = ((int64_t)d.nb << d.nsig) / WPB;
  const int64_t per = (rounds + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < rounds ? lo + per : rounds;
  const int na = 1 << d.a, nc = 1 << d.c;
  const int64_t sig_mask = (int64_t(1) << d.nsig) - 1;
  float2 pre[kInPer];
  auto prefetch = [&](int64_t it) {
    const float2* src = d.X0 + (it >> d.nsig) * d.sX0 + ((it & sig_mask) << d.a);
#pragma unroll
    for (int i = 0; i < kInPer; ++i) {
      const int e = lane + 64 * i;
      if (e < na) pre[i] = src[e];
    }
  };
  if (lo < hi) prefetch(lo * WPB + wave);
  int64_t cur_b = -1;
  float vmax = 0.f;
  __syncthreads();  // tables
  for (int64_t r = lo; r < hi; ++r) {
    const int64_t it = r * WPB + wave;
    const int64_t b = it >> d.nsig, sig = it & sig_mask;
    if (b != cur_b) {  // the same for every wave of the block
      if (d.scale_c && cur_b >= 0) {
        float v = vmax;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
        if (lane == 0) raise_max(d.scale_c + cur_b, v);
        vmax = 0.f;
      }
      __syncthreads();  // every wave is done with the previous slice's tensors
      for (int j = 0; j < d.nstages; ++j) {
        const FusedStage& s = d.st[j];
        const float2* y = s.Y + b * s.sY;
        const int ny = 1 << (s.k + s.n);
        for (int e = tid; e < ny; e += 64 * WPB) Ys[s.yoff + e] = y[e];
      }
      __syncthreads();
      cur_b = b;
    }
#pragma unroll
    for (int i = 0; i < kInPer; ++i) {
      const int e = lane + 64 * i;
      if (e < na) buf0[e] = pre[i];
    }
    if (r + 1 < hi) prefetch(it + WPB);
    __syncwarp();
    float2* in = buf0;
    float2* out = buf1;
    for (int j = 0; j < d.nstages; ++j) {
      const FusedStage& s = d.st[j];
      const int K = 1 << s.k;
      // register blocks of RB rows x NB columns, as large as 4 x 4 while
      // every lane keeps a block (2^(m+n) / (RB NB) >= 64)
      int bb = s.m + s.n - 6;
      bb = bb < 0 ? 0 : (bb > 4 ? 4 : bb);
      int rbits = (bb + 1) / 2;
      rbits = rbits > s.m ? s.m : rbits;
      int nbits = bb - rbits;
      nbits = nbits > s.n ? s.n : nbits;
      rbits = bb - nbits > s.m ? s.m : bb - nbits;
      const int code = (rbits << 2) | nbits;
      const float2* yb = Ys + s.yoff;
      switch (code) {
        case (2 << 2) | 2: stage_k<4, 4>(in, out, yb, s.k, s.m, s.n, rbits, nbits, rowP[j], nP[j], lane); break;
        case (2 << 2) | 1: stage_k<4, 2>(in, out, yb, s.k, s.m, s.n, rbits, nbits, rowP[j], nP[j], lane); break;
        case (1 << 2) | 2: stage_k<2, 4>(in, out, yb, s.k, s.m, s.n, rbits, nbits, rowP[j], nP[j], lane); break;
        case (1 << 2) | 1: stage_k<2, 2>(in, out, yb, s.k, s.m, s.n, rbits, nbits, rowP[j], nP[j], lane); break;
        case (2 << 2) | 0: stage_k<4, 1>(in, out, yb, s.k, s.m, s.n, rbits, nbits, rowP[j], nP[j], lane); break;
        case (0 << 2) | 2: stage_k<1, 4>(in, out, yb, s.k, s.m, s.n, rbits, nbits, rowP[j], nP[j], lane); break;
        case (1 << 2) | 0: stage_k<2, 1>(in, out, yb, s.k, s.m, s.n, rbits, nbits, rowP[j], nP[j], lane); break;
        case (0 << 2) | 1: stage_k<1, 2>(in, out, yb, s.k, s.m, s.n, rbits, nbits, rowP[j], nP[j], lane); break;
        default: stage_k<1, 1>(in, out, yb, s.k, s.m, s.n, rbits, nbits, rowP[j], nP[j], lane); break;
      }
      __syncwarp();
      float2* tmp = in;
      in = out;
      out = tmp;
    }
    float2* dst = d.XL + b * d.sXL + pdep_f((uint64_t)sig, d.sig_out);
    for (int w = lane; w < nc; w += 64) {
      const float2 v = in[w];
      dst[wT[w & 63] | wT[64 + (w >> 6)]] = v;
      vmax = fmaxf(vmax, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    __syncwarp();  // the next piece overwrites buf0
  }
  if (d.scale_c && cur_b >= 0) {
    float v = vmax;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if (lane == 0) raise_max(d.scale_c + cur_b, v);
  }
}

}  // namespace

void launch_fused(const FusedDesc& d, hipStream_t st) {
  // waves per block: as many as keep two working buffers per wave plus the
  // small tensors within 64 KiB of LDS
  const int wpb = d.rmax <= 9 ? 4 : (d.rmax == 10 ? 2 : 1);
  const int64_t rounds = ((int64_t)d.nb << d.nsig) / wpb;
  const int blocks = (int)(rounds < 2048 ? rounds : 2048);
  const size_t lds = ((size_t)wpb * 2 * ((size_t)1 << d.rmax) + (size_t)d.y_elems) * sizeof(float2);
  switch (wpb) {
    case 4:
      hipLaunchKernelGGL(k_fused<4>, dim3(blocks), dim3(256), lds, st, d);
      break;
    case 2:
      hipLaunchKernelGGL(k_fused<2>, dim3(blocks), dim3(128), lds, st, d);
      break;
    default:
      hipLaunchKernelGGL(k_fused<1>, dim3(blocks), dim3(64), lds, st, d);
      break;
  }
}

}  // namespace ltn
