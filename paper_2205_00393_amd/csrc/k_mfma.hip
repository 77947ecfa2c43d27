// Complex GEMM of one contraction step on CDNA4 matrix cores.
//
//   C[merge(m, n)] = sum_k A[m * K + k] * B[n * K + k]     (complex64)
//
// Both operands keep the contracted index innermost (the plan's layout
// rule), so this is an "NT" GEMM. A complex product is run as a real GEMM
// of size M x 2N x 2K: A is used as stored (re, im interleaved along k) and
// each complex b of B becomes the real 2x2 block [[br, -bi], [bi, br]]
// (rows: output re / im, columns: input re / im), built while B is read
// from LDS. The real output [M][2N] is then complex C[m][n] interleaved.
//
// v_mfma_f32_32x32x2_f32 consumes, per lane l, A[l % 32][l / 32] and
// B[l / 32][l % 32]; lane l holds C[8 g + 4 (l / 32) + q][l % 32] in
// accumulator 4 g + q. Two MFMAs cover two complex k per step: the first
// takes the real parts of A (k and k+1 on the two half-waves), the second
// the imaginary parts.
//
// Split precision (k_cgemm_split): every real part x of an operand is
// scaled by an exact power of two sigma (from the operand's largest
// magnitude, recorded by its producer) and split as x sigma = hi + 2^-s lo
// with hi, lo in fp16 (s = 11) or bf16 (s = 8). With hi' = 2^s hi (exact),
//     2^s (x sigma_x)(y sigma_y) ~ hi'_x hi_y + hi_x lo_y + lo_x hi_y
// (lo lo dropped), so three v_mfma_f32_32x32x16_{f16,bf16} per tile feed
// one FP32 accumulator, rescaled by 2^-s / (sigma_A sigma_B) at the end.
// Each lane supplies 8 consecutive k' = 2 k + (re|im) values of a row of A
// as stored, and of B in the 2x2 real form: (re, -im) pairs for output
// real parts, (im, re) pairs for imaginary parts (sign flip / half swap).
#include "kernels.h"

namespace ltn {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint64_t pdep64(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  while (mask && x) {
    uint64_t low = mask & (~mask + 1);
    if (x & 1) r |= low;
    x >>= 1;
    mask &= mask - 1;
  }
  return r;
}

// wave-wide max, then one atomic per wave: the largest |x| of a tensor slice
// (non-negative floats order like their bit patterns)
__device__ __forceinline__ void record_max(uint32_t* slot, float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0 && v > 0.f) atomicMax(slot, __float_as_uint(v));
}

// sigma = 2^(-floor(log2 max)), so that max * sigma lies in [1, 2)
__device__ __forceinline__ float scale_of(uint32_t maxbits) {
  int e = (int)((maxbits >> 23) & 0xff);
  if (e == 0 || e == 0xff) return 1.f;
  int se = 254 - e;  // biased exponent of 2^(127 - e)
  if (se < 1) se = 1;
  if (se > 254) se = 254;
  return __uint_as_float((uint32_t)se << 23);
}

template <int BM, int BNC, int BKC>
struct Cfg {
  static constexpr int WM = BM / 2;          // rows per wave
  static constexpr int TM = WM / 32;         // 32-row MFMA tiles per wave
  static constexpr int WNC = BNC / 2;        // complex columns per wave
  static constexpr int TN = (2 * WNC) / 32;  // 32-real-column MFMA tiles per wave
  static constexpr int LDA = BKC + 1;        // padded row length (complex)
  static constexpr int CHA = BM * BKC / 2;   // float4 chunks of the A tile
  static constexpr int CHB = BNC * BKC / 2;
  static constexpr int RA = (CHA + 255) / 256;
  static constexpr int RB = (CHB + 255) / 256;
  static_assert(TM >= 1 && TN >= 1 && BKC >= 2, "tile too small");
};

template <int BM, int BNC, int BKC>
__global__ __launch_bounds__(256) void k_cgemm_c64(GemmDesc d) {
  using C = Cfg<BM, BNC, BKC>;
  __shared__ float2 As[BM * C::LDA];
  __shared__ float2 Bs[BNC * C::LDA];

  const int64_t M = int64_t(1) << d.m, N = int64_t(1) << d.n, K = int64_t(1) << d.k;
  const int tiles_n = (int)(N / BNC);
  const int64_t tiles = (M / BM) * tiles_n;
  const int64_t total = tiles * d.nb;
  // XCD-aware order: consecutive logical tiles (sharing an A panel) land on
  // the same XCD, whose L2 then serves the panel to all of them
  int64_t w = blockIdx.x;
  int64_t logical = (total % 8 == 0) ? (w % 8) * (total / 8) + w / 8 : w;
  const int64_t b = logical / tiles;
  const int64_t t = logical % tiles;
  const int64_t bm = t / tiles_n, bn = t % tiles_n;

  const float2* A = d.A + b * d.sA + bm * BM * K;
  const float2* B = d.B + b * d.sB + bn * BNC * K;
  float* Cf = reinterpret_cast<float*>(d.C + b * d.sC);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, i = lane & 31;

  floatx16 acc[C::TM][C::TN];
#pragma unroll
  for (int x = 0; x < C::TM; ++x)
#pragma unroll
    for (int y = 0; y < C::TN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.f;

  float4 ra[C::RA], rb[C::RB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < C::RA; ++r) {
      int c = tid + 256 * r;
      if (c < C::CHA) {
        int row = c / (BKC / 2), col = c % (BKC / 2);
        ra[r] = *reinterpret_cast<const float4*>(A + row * K + k0 + 2 * col);
      }
    }
#pragma unroll
    for (int r = 0; r < C::RB; ++r) {
      int c = tid + 256 * r;
      if (c < C::CHB) {
        int row = c / (BKC / 2), col = c % (BKC / 2);
        rb[r] = *reinterpret_cast<const float4*>(B + row * K + k0 + 2 * col);
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int r = 0; r < C::RA; ++r) {
      int c = tid + 256 * r;
      if (c < C::CHA) {
        int row = c / (BKC / 2), col = c % (BKC / 2);
        As[row * C::LDA + 2 * col] = make_float2(ra[r].x, ra[r].y);
        As[row * C::LDA + 2 * col + 1] = make_float2(ra[r].z, ra[r].w);
      }
    }
#pragma unroll
    for (int r = 0; r < C::RB; ++r) {
      int c = tid + 256 * r;
      if (c < C::CHB) {
        int row = c / (BKC / 2), col = c % (BKC / 2);
        Bs[row * C::LDA + 2 * col] = make_float2(rb[r].x, rb[r].y);
        Bs[row * C::LDA + 2 * col + 1] = make_float2(rb[r].z, rb[r].w);
      }
    }
  };

  const int arow0 = wm * C::WM + i;
  // B column of this lane in MFMA tile y: real column 32 y + i of the wave
  // = complex column (32 y + i) / 2, part i & 1 (0: re, 1: im)
  const int bcol0 = wn * C::WNC + (i >> 1);
  const bool im_col = (i & 1) != 0;

  load(0);
  for (int64_t k0 = 0; k0 < K; k0 += BKC) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + BKC < K) load(k0 + BKC);
#pragma unroll
    for (int kp = 0; kp < BKC; kp += 2) {
      float2 av[C::TM], bv[C::TN];
#pragma unroll
      for (int x = 0; x < C::TM; ++x) av[x] = As[(arow0 + 32 * x) * C::LDA + kp + h];
#pragma unroll
      for (int y = 0; y < C::TN; ++y) bv[y] = Bs[(bcol0 + 16 * y) * C::LDA + kp + h];
#pragma unroll
      for (int y = 0; y < C::TN; ++y) {
        float b1 = im_col ? bv[y].y : bv[y].x;   // pairs with Re a
        float b2 = im_col ? bv[y].x : -bv[y].y;  // pairs with Im a
#pragma unroll
        for (int x = 0; x < C::TM; ++x) {
          acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[x].x, b1, acc[x][y], 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[x].y, b2, acc[x][y], 0, 0, 0);
        }
      }
    }
  }

  // epilogue: pdep is additive over disjoint bit groups of the row index
  const uint64_t maskA = d.cmask;
  const uint64_t maskB = ~d.cmask & ((1ull << (d.m + d.n)) - 1);
  const uint64_t row_base = (uint64_t)(bm * BM + wm * C::WM + 4 * h);
  const uint64_t pbase = pdep64(row_base, maskA);
  uint64_t pq[4], pg[4], pt[C::TM];
#pragma unroll
  for (int q = 0; q < 4; ++q) pq[q] = pdep64((uint64_t)q, maskA);
#pragma unroll
  for (int g = 0; g < 4; ++g) pg[g] = pdep64((uint64_t)(8 * g), maskA);
#pragma unroll
  for (int x = 0; x < C::TM; ++x) pt[x] = pdep64((uint64_t)(32 * x), maskA);
  float vmax = 0.f;
#pragma unroll
  for (int y = 0; y < C::TN; ++y) {
    uint64_t ncol = (uint64_t)(bn * BNC + bcol0 + 16 * y);
    uint64_t pn = pdep64(ncol, maskB);
#pragma unroll
    for (int x = 0; x < C::TM; ++x)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint64_t addr = pbase | pt[x] | pg[g] | pq[q] | pn;
          float v = acc[x][y][4 * g + q];
          vmax = fmaxf(vmax, fabsf(v));
          Cf[2 * addr + (im_col ? 1 : 0)] = v;
        }
  }
  if (d.scale_c) record_max(d.scale_c + b, vmax);
}


template <bool BF>
struct SplitType;
template <>
struct SplitType<false> {
  using T = _Float16;
  typedef _Float16 V8 __attribute__((ext_vector_type(8)));
  static constexpr int S = 11;
};
template <>
struct SplitType<true> {
  using T = __bf16;
  typedef __bf16 V8 __attribute__((ext_vector_type(8)));
  static constexpr int S = 8;
};

template <bool BF>
__device__ __forceinline__ floatx16 mfma16(uint4 a, uint4 b, floatx16 c) {
  if constexpr (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(typename SplitType<true>::V8, a),
                                                   __builtin_bit_cast(typename SplitType<true>::V8, b),
                                                   c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(typename SplitType<false>::V8, a),
                                                  __builtin_bit_cast(typename SplitType<false>::V8, b),
                                                  c, 0, 0, 0);
}

// x -> (hi, lo) of x * sigma, and hi * 2^s
template <bool BF>
__device__ __forceinline__ void split1(float v, float sigma, uint16_t& hi, uint16_t& hs, uint16_t& lo) {
  using T = typename SplitType<BF>::T;
  constexpr float P = (float)(1 << SplitType<BF>::S);
  float x = v * sigma;
  T h = (T)x;
  float hf = (float)h;
  T l = (T)((x - hf) * P);
  T hsv = (T)(hf * P);
  hi = __builtin_bit_cast(uint16_t, h);
  lo = __builtin_bit_cast(uint16_t, l);
  hs = __builtin_bit_cast(uint16_t, hsv);
}

// B operand of output real parts: (re, -im) pairs; imaginary parts: (im, re)
__device__ __forceinline__ uint4 bform(uint4 w, bool im_col) {
  if (im_col) {
    w.x = (w.x << 16) | (w.x >> 16);
    w.y = (w.y << 16) | (w.y >> 16);
    w.z = (w.z << 16) | (w.z >> 16);
    w.w = (w.w << 16) | (w.w >> 16);
  } else {
    w.x ^= 0x80000000u;
    w.y ^= 0x80000000u;
    w.z ^= 0x80000000u;
    w.w ^= 0x80000000u;
  }
  return w;
}

template <int BM, int BNC, int BKC, bool BF>
__global__ __launch_bounds__(256) void k_cgemm_split(GemmDesc d) {
  using C = Cfg<BM, BNC, BKC>;
  constexpr int LDK = 2 * BKC + 8;  // halves per LDS row (16-byte pad)
  static_assert(BKC % 8 == 0, "split tiles need 8 complex k per MFMA");
  __shared__ uint16_t Ahi[BM * LDK], Alo[BM * LDK];
  __shared__ uint16_t Bhi[BNC * LDK], Bhs[BNC * LDK], Blo[BNC * LDK];

  const int64_t M = int64_t(1) << d.m, N = int64_t(1) << d.n, K = int64_t(1) << d.k;
  const int tiles_n = (int)(N / BNC);
  const int64_t tiles = (M / BM) * tiles_n;
  const int64_t total = tiles * d.nb;
  int64_t w = blockIdx.x;
  int64_t logical = (total % 8 == 0) ? (w % 8) * (total / 8) + w / 8 : w;
  const int64_t b = logical / tiles;
  const int64_t t = logical % tiles;
  const int64_t bm = t / tiles_n, bn = t % tiles_n;

  const float sa = scale_of(d.scale_a[b]), sb = scale_of(d.scale_b[b]);
  const float2* A = d.A + b * d.sA + bm * BM * K;
  const float2* B = d.B + b * d.sB + bn * BNC * K;
  float* Cf = reinterpret_cast<float*>(d.C + b * d.sC);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, i = lane & 31;

  floatx16 acc[C::TM][C::TN];
#pragma unroll
  for (int x = 0; x < C::TM; ++x)
#pragma unroll
    for (int y = 0; y < C::TN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.f;

  float4 ra[C::RA], rb[C::RB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < C::RA; ++r) {
      int c = tid + 256 * r;
      if (c < C::CHA) {
        int row = c / (BKC / 2), col = c % (BKC / 2);
        ra[r] = *reinterpret_cast<const float4*>(A + row * K + k0 + 2 * col);
      }
    }
#pragma unroll
    for (int r = 0; r < C::RB; ++r) {
      int c = tid + 256 * r;
      if (c < C::CHB) {
        int row = c / (BKC / 2), col = c % (BKC / 2);
        rb[r] = *reinterpret_cast<const float4*>(B + row * K + k0 + 2 * col);
      }
    }
  };
  auto pack2 = [](uint16_t a, uint16_t b2) { return (uint32_t)a | ((uint32_t)b2 << 16); };
  auto stash = [&]() {
#pragma unroll
    for (int r = 0; r < C::RA; ++r) {
      int c = tid + 256 * r;
      if (c < C::CHA) {
        int row = c / (BKC / 2), col = c % (BKC / 2);
        uint16_t h0, h1, h2, h3, s0, s1, s2, s3, l0, l1, l2, l3;
        split1<BF>(ra[r].x, sa, h0, s0, l0);
        split1<BF>(ra[r].y, sa, h1, s1, l1);
        split1<BF>(ra[r].z, sa, h2, s2, l2);
        split1<BF>(ra[r].w, sa, h3, s3, l3);
        int o = row * LDK + 4 * col;
        *reinterpret_cast<uint2*>(&Ahi[o]) = make_uint2(pack2(h0, h1), pack2(h2, h3));
        *reinterpret_cast<uint2*>(&Alo[o]) = make_uint2(pack2(l0, l1), pack2(l2, l3));
      }
    }
#pragma unroll
    for (int r = 0; r < C::RB; ++r) {
      int c = tid + 256 * r;
      if (c < C::CHB) {
        int row = c / (BKC / 2), col = c % (BKC / 2);
        uint16_t h0, h1, h2, h3, s0, s1, s2, s3, l0, l1, l2, l3;
        split1<BF>(rb[r].x, sb, h0, s0, l0);
        split1<BF>(rb[r].y, sb, h1, s1, l1);
        split1<BF>(rb[r].z, sb, h2, s2, l2);
        split1<BF>(rb[r].w, sb, h3, s3, l3);
        int o = row * LDK + 4 * col;
        *reinterpret_cast<uint2*>(&Bhi[o]) = make_uint2(pack2(h0, h1), pack2(h2, h3));
        *reinterpret_cast<uint2*>(&Bhs[o]) = make_uint2(pack2(s0, s1), pack2(s2, s3));
        *reinterpret_cast<uint2*>(&Blo[o]) = make_uint2(pack2(l0, l1), pack2(l2, l3));
      }
    }
  };

  const int arow0 = wm * C::WM + i;
  const int bcol0 = wn * C::WNC + (i >> 1);
  const bool im_col = (i & 1) != 0;

  load(0);
  for (int64_t k0 = 0; k0 < K; k0 += BKC) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + BKC < K) load(k0 + BKC);
#pragma unroll
    for (int ch = 0; ch < BKC / 8; ++ch) {
      const int ko = 16 * ch + 8 * h;  // halves offset of this lane's 8 k'
      uint4 ah[C::TM], al[C::TM];
#pragma unroll
      for (int x = 0; x < C::TM; ++x) {
        int o = (arow0 + 32 * x) * LDK + ko;
        ah[x] = *reinterpret_cast<const uint4*>(&Ahi[o]);
        al[x] = *reinterpret_cast<const uint4*>(&Alo[o]);
      }
#pragma unroll
      for (int y = 0; y < C::TN; ++y) {
        int o = (bcol0 + 16 * y) * LDK + ko;
        uint4 bh = bform(*reinterpret_cast<const uint4*>(&Bhi[o]), im_col);
        uint4 bs = bform(*reinterpret_cast<const uint4*>(&Bhs[o]), im_col);
        uint4 bl = bform(*reinterpret_cast<const uint4*>(&Blo[o]), im_col);
#pragma unroll
        for (int x = 0; x < C::TM; ++x) {
          acc[x][y] = mfma16<BF>(ah[x], bs, acc[x][y]);
          acc[x][y] = mfma16<BF>(ah[x], bl, acc[x][y]);
          acc[x][y] = mfma16<BF>(al[x], bh, acc[x][y]);
        }
      }
    }
  }

  const float post = (1.0f / (float)(1 << SplitType<BF>::S)) / sa / sb;
  const uint64_t maskA = d.cmask;
  const uint64_t maskB = ~d.cmask & ((1ull << (d.m + d.n)) - 1);
  const uint64_t row_base = (uint64_t)(bm * BM + wm * C::WM + 4 * h);
  const uint64_t pbase = pdep64(row_base, maskA);
  uint64_t pq[4], pg[4], pt[C::TM];
#pragma unroll
  for (int q = 0; q < 4; ++q) pq[q] = pdep64((uint64_t)q, maskA);
#pragma unroll
  for (int g = 0; g < 4; ++g) pg[g] = pdep64((uint64_t)(8 * g), maskA);
#pragma unroll
  for (int x = 0; x < C::TM; ++x) pt[x] = pdep64((uint64_t)(32 * x), maskA);
  float vmax = 0.f;
#pragma unroll
  for (int y = 0; y < C::TN; ++y) {
    uint64_t ncol = (uint64_t)(bn * BNC + bcol0 + 16 * y);
    uint64_t pn = pdep64(ncol, maskB);
#pragma unroll
    for (int x = 0; x < C::TM; ++x)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint64_t addr = pbase | pt[x] | pg[g] | pq[q] | pn;
          float v = acc[x][y][4 * g + q] * post;
          vmax = fmaxf(vmax, fabsf(v));
          Cf[2 * addr + (im_col ? 1 : 0)] = v;
        }
  }
  if (d.scale_c) record_max(d.scale_c + b, vmax);
}

struct CfgInfo {
  int bm, bnc, bkc;
  const char* name;
};
const CfgInfo kCfgs[] = {
    {128, 64, 16, "c64_128x64x16"}, {64, 64, 16, "c64_64x64x16"},  {128, 32, 16, "c64_128x32x16"},
    {64, 32, 16, "c64_64x32x16"},   {128, 64, 8, "c64_128x64x8"},  {64, 32, 8, "c64_64x32x8"},
    {64, 32, 4, "c64_64x32x4"},     {64, 32, 2, "c64_64x32x2"},    {256, 64, 16, "c64_256x64x16"},
    {128, 128, 16, "c64_128x128x16"},
};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
const CfgInfo kSplitCfgs[] = {
    {256, 64, 16, "split_256x64x16"}, {128, 64, 16, "split_128x64x16"}, {128, 128, 16, "split_128x128x16"},
    {128, 32, 16, "split_128x32x16"}, {64, 64, 16, "split_64x64x16"},   {64, 32, 16, "split_64x32x16"},
    {128, 64, 8, "split_128x64x8"},   {64, 32, 8, "split_64x32x8"},
};
constexpr int kNumSplit = sizeof(kSplitCfgs) / sizeof(kSplitCfgs[0]);

template <int BM, int BNC, int BKC>
void run(const GemmDesc& d, hipStream_t st) {
  int64_t tiles = ((int64_t(1) << d.m) / BM) * ((int64_t(1) << d.n) / BNC) * d.nb;
  hipLaunchKernelGGL((k_cgemm_c64<BM, BNC, BKC>), dim3((unsigned)tiles), dim3(256), 0, st, d);
}

template <int BM, int BNC, int BKC>
void run_split(const GemmDesc& d, bool bf, hipStream_t st) {
  int64_t tiles = ((int64_t(1) << d.m) / BM) * ((int64_t(1) << d.n) / BNC) * d.nb;
  if (bf)
    hipLaunchKernelGGL((k_cgemm_split<BM, BNC, BKC, true>), dim3((unsigned)tiles), dim3(256), 0, st, d);
  else
    hipLaunchKernelGGL((k_cgemm_split<BM, BNC, BKC, false>), dim3((unsigned)tiles), dim3(256), 0, st, d);
}

const CfgInfo& info_of(int cfg, int mode) { return mode == LTN_C64 ? kCfgs[cfg] : kSplitCfgs[cfg]; }

}  // namespace

int gemm_config_count(int mode) { return mode == LTN_C64 ? kNumCfgs : kNumSplit; }

bool gemm_config_fits(int cfg, int m, int k, int n, int mode) {
  if (cfg < 0 || cfg >= gemm_config_count(mode)) return false;
  const CfgInfo& c = info_of(cfg, mode);
  return m < 40 && n < 40 && (1ll << m) >= c.bm && (1ll << n) >= c.bnc && (1ll << k) >= c.bkc;
}

const char* gemm_config_name(int cfg, int mode) {
  return cfg >= 0 && cfg < gemm_config_count(mode) ? info_of(cfg, mode).name : "?";
}

void launch_cgemm(const GemmDesc& d, int mode, hipStream_t st) {
  if (mode != LTN_C64) {
    bool bf = mode == LTN_SPLIT_BF16;
    switch (d.cfg) {
      case 0: run_split<256, 64, 16>(d, bf, st); break;
      case 1: run_split<128, 64, 16>(d, bf, st); break;
      case 2: run_split<128, 128, 16>(d, bf, st); break;
      case 3: run_split<128, 32, 16>(d, bf, st); break;
      case 4: run_split<64, 64, 16>(d, bf, st); break;
      case 5: run_split<64, 32, 16>(d, bf, st); break;
      case 6: run_split<128, 64, 8>(d, bf, st); break;
      case 7: run_split<64, 32, 8>(d, bf, st); break;
    }
    return;
  }
  switch (d.cfg) {
    case 0: run<128, 64, 16>(d, st); break;
    case 1: run<64, 64, 16>(d, st); break;
    case 2: run<128, 32, 16>(d, st); break;
    case 3: run<64, 32, 16>(d, st); break;
    case 4: run<128, 64, 8>(d, st); break;
    case 5: run<64, 32, 8>(d, st); break;
    case 6: run<64, 32, 4>(d, st); break;
    case 7: run<64, 32, 2>(d, st); break;
    case 8: run<256, 64, 16>(d, st); break;
    case 9: run<128, 128, 16>(d, st); break;
  }
}

}  // namespace ltn
