// Complex GEMM of one contraction step on CDNA4 matrix cores.
//
//   C[merge(m, n)] = sum_k A[m * K + k] * B[n * K + k]     (complex64)
//
// Both operands keep the contracted index innermost (the plan's layout
// rule), so this is an "NT" GEMM. The direct tiles run a complex product
// as a real GEMM of size M x 2N x 2K; the three-product tiles as three
// real GEMMs of M x N x K (see k_cgemm_c64). In the direct form A is used
// as stored (re, im interleaved along k) and each complex b of B becomes
// the real 2x2 block [[br, -bi], [bi, br]] (rows: output re / im, columns:
// input re / im), built while B is read from LDS. The real output [M][2N]
// is then complex C[m][n] interleaved.
//
// v_mfma_f32_32x32x2_f32 consumes, per lane l, A[l % 32][l / 32] and
// B[l / 32][l % 32]; lane l holds C[8 g + 4 (l / 32) + q][l % 32] in
// accumulator 4 g + q. Two MFMAs cover two complex k per step: the first
// takes the real parts of A (k and k+1 on the two half-waves), the second
// the imaginary parts.
//
// Split precision. Before a split step, k_split_convert writes a copy of
// each operand in the split layout: every group of 4 consecutive
// complex elements (32 bytes) becomes 16 bytes of hi parts then 16 bytes of
// lo parts, (re, im) interleaved. fp16: x sigma = hi + 2^-11 lo with sigma an
// exact power of two from the operand's largest magnitude (recorded by its
// producer), so hi and lo stay in fp16's normal range; bf16 shares FP32's
// exponent range and needs no scale: x = hi + lo. k_cgemm_split then sums
// hi*hi, hi*lo and lo*hi (lo*lo dropped) with v_mfma_f32_32x32x16_{f16,bf16}
// into one FP32 accumulator (fp16: the hi*hi product uses hi * 2^11, exact,
// so all three terms share the accumulator's scale) and undoes the scaling
// in the epilogue. Each lane supplies 8 consecutive k' = 2 k + (re|im) of a
// row of A as stored, and of B in the 2x2 real form: (re, -im) pairs for
// output real parts, (im, re) pairs for imaginary parts (sign flip / half
// swap of each 32-bit word).
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
  if ((threadIdx.x & 63) == 0) raise_max(slot, v);
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

// Block -> (slice, row tile, column tile). Hardware dispatch sends block w to
// XCD w % 8, so each XCD first gets a contiguous 1/8 of the logical tiles;
// inside a slice, tiles go in groups of G = 8 row tiles, column-major within a
// group, so the blocks resident at once share both row and column panels in
// their XCD's L2 (operand re-reads ~ A / G_n + B / G_m instead of B per row).
__device__ __forceinline__ void tile_of(int64_t w, int64_t tiles_m, int64_t tiles_n, int nb,
                                        int64_t& b, int64_t& bm, int64_t& bn) {
  const int64_t tiles = tiles_m * tiles_n, total = tiles * nb;
  const int64_t logical = (total % 8 == 0) ? (w % 8) * (total / 8) + w / 8 : w;
  b = logical / tiles;
  const int64_t t = logical % tiles;
  const int64_t G = tiles_m < 8 ? tiles_m : 8;
  const int64_t grp = t / (G * tiles_n), r = t % (G * tiles_n);
  bm = grp * G + r % G;
  bn = r / G;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

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
  static constexpr int S = 0;
};

template <bool BF>
__device__ __forceinline__ uint32_t split_pair(float a, float b, float sigma, uint32_t& lo) {
  using T = typename SplitType<BF>::T;
  constexpr float P = (float)(1 << SplitType<BF>::S);
  float xa = a * sigma, xb = b * sigma;
  T ha = (T)xa, hb = (T)xb;
  T la = (T)((xa - (float)ha) * P), lb = (T)((xb - (float)hb) * P);
  lo = (uint32_t)__builtin_bit_cast(uint16_t, la) | ((uint32_t)__builtin_bit_cast(uint16_t, lb) << 16);
  return (uint32_t)__builtin_bit_cast(uint16_t, ha) | ((uint32_t)__builtin_bit_cast(uint16_t, hb) << 16);
}

// One complex output written in the split layout (groups of 4 consecutive
// complex: 16 bytes of hi words, then 16 bytes of lo words; a word holds
// (re, im)); the same bits as the conversion pass produces with scale sigma.
template <bool BF>
__device__ __forceinline__ void store_split(uint32_t* Cw, uint64_t addr, float re, float im, float sigma) {
  uint32_t lo;
  const uint32_t hi = split_pair<BF>(re, im, sigma, lo);
  uint32_t* g = Cw + (addr >> 2) * 8 + (addr & 3);
  g[0] = hi;
  g[4] = lo;
}

// Scale of an fp16 split output written by its producer: from the bound
// |Re c|, |Im c| <= |c| <= K max|a| max|b| <= 2 K max|Re, Im a| max|Re, Im b|
// (the output's own maximum is not known before it is written). One thread
// stores the bound for the consumer, which derives the same scale from it.
__device__ __forceinline__ float split_out_scale(const GemmDesc& d, int64_t b, int64_t K, bool store) {
  const float bound = 2.f * (float)K * __uint_as_float(d.max_a[b]) * __uint_as_float(d.max_b[b]);
  if (store) d.bound_c[b] = __float_as_uint(bound);
  return scale_of(__float_as_uint(bound));
}

// NWN waves along the columns (2: waves 2 x 2; 1: waves 4 x 1, for tiles
// of 16 complex columns). G3: the three-product form, whose MFMA columns
// are complex outputs (32 per tile) instead of real ones (16 complex).
template <int BM, int BNC, int BKC, int NWN = 2, bool G3 = false>
struct Cfg {
  static constexpr int WM = BM / (4 / NWN);  // rows per wave
  static constexpr int TM = WM / 32;         // 32-row MFMA tiles per wave
  static constexpr int WNC = BNC / NWN;      // complex columns per wave
  static constexpr int CPT = G3 ? 32 : 16;   // complex columns per MFMA tile
  static constexpr int TN = WNC / CPT;       // MFMA column tiles per wave
  static constexpr int LDA = BKC + 1;        // padded row length (complex)
  static constexpr int CHA = BM * BKC / 2;   // float4 chunks of the A tile
  static constexpr int CHB = BNC * BKC / 2;
  static constexpr int RA = (CHA + 255) / 256;
  static constexpr int RB = (CHB + 255) / 256;
  static_assert(TM >= 1 && TN >= 1 && BKC >= 2, "tile too small");
};

// SPLITK: block w takes chunk w / (tiles * nb) of the sum (2^kc_bits
// consecutive k) for tile w % (tiles * nb), and writes its FP32 partial of
// C to part in plain row-major order ([b][chunk][row][column]); the split
// layout and the per-slice maxima are left to the pass that adds the chunks.
//
// G3: the complex product by three real products (Gauss's method; its
// rounding for matrix products is analysed by Higham, SIAM J. Matrix Anal.
// Appl. 13, 1992):
//   P1 = Ar Br^T,  P2 = Ai Bi^T,  P3 = (Ar + Ai)(Br + Bi)^T,
//   Re C = P1 - P2,  Im C = P3 - P1 - P2,
// three real GEMMs of M x N x K, i.e. 3 real MACs per complex MAC instead
// of the 4 of the 2x2 real form. The real part's error bound has the form
// of the direct form's (two sums and a subtraction instead of one sum of
// both); the imaginary part's grows from terms in |Ar||Bi| + |Ai||Br| to
// terms in (|Ar| + |Ai|)(|Br| + |Bi|), at most about twice as large. Lane l's MFMA operand is row l % 32, k l / 32 of A
// and column l % 32 of B, so one 8-byte LDS read of a complex element of
// each gives the operands of P1 and P2, and their sums those of P3; the
// accumulators of a lane hold whole complex outputs.
//
// MINW: waves per SIMD the registers must allow (1: the compiler's choice;
// the three-product 128 x 64 x 16 tile fits three with its accumulators in
// VGPRs and no spills, against two when left to the compiler).
template <int BM, int BNC, int BKC, int NWN = 2, bool SPLITK = false, bool G3 = false, int MINW = 1>
__global__ __launch_bounds__(256, MINW) void k_cgemm_c64(GemmDesc d) {
  using C = Cfg<BM, BNC, BKC, NWN, G3>;
  __shared__ float2 As[BM * C::LDA];
  __shared__ float2 Bs[BNC * C::LDA];

  const int64_t M = int64_t(1) << d.m, N = int64_t(1) << d.n, K = int64_t(1) << d.k;
  int64_t b, bm, bn, chunk = 0, w = blockIdx.x;
  if constexpr (SPLITK) {
    const int64_t per = (M / BM) * (N / BNC) * d.nb;
    chunk = w / per;
    w -= chunk * per;
  }
  tile_of(w, M / BM, N / BNC, d.nb, b, bm, bn);
  const int64_t KL = SPLITK ? (int64_t(1) << d.kc_bits) : K;  // sum length of this block
  const int64_t k_first = chunk * KL;

  const float2* A = d.A + b * d.sA + bm * BM * K + k_first;
  const float2* B = d.B + b * d.sB + bn * BNC * K + k_first;
  float* Cf = SPLITK ? reinterpret_cast<float*>(d.part + ((b << (d.k - d.kc_bits)) + chunk) * (M * N))
                     : reinterpret_cast<float*>(d.C + b * d.sC);
  const float so = !SPLITK && d.split_out == 2 ? split_out_scale(d, b, K, bm == 0 && bn == 0 && threadIdx.x == 0) : 1.f;
  uint32_t* Cw = reinterpret_cast<uint32_t*>(d.C + b * d.sC);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const int h = lane >> 5, i = lane & 31;

  // G3: acc = P1, acc2 = P2, acc3 = P3 (unused by the direct form)
  constexpr int T2 = G3 ? C::TM : 1, U2 = G3 ? C::TN : 1;
  floatx16 acc[C::TM][C::TN], acc2[T2][U2], acc3[T2][U2];
#pragma unroll
  for (int x = 0; x < C::TM; ++x)
#pragma unroll
    for (int y = 0; y < C::TN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.f;
#pragma unroll
  for (int x = 0; x < T2; ++x)
#pragma unroll
    for (int y = 0; y < U2; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc2[x][y][v] = 0.f;
        acc3[x][y][v] = 0.f;
      }

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
  // B column of this lane in MFMA tile y: direct form: real column 32 y + i
  // of the wave = complex column (32 y + i) / 2, part i & 1 (0: re, 1: im);
  // G3: complex column 32 y + i
  const int bcol0 = wn * C::WNC + (G3 ? i : (i >> 1));
  const bool im_col = !G3 && (i & 1) != 0;

  load(0);
  for (int64_t k0 = 0; k0 < KL; k0 += BKC) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + BKC < KL) load(k0 + BKC);
#pragma unroll
    for (int kp = 0; kp < BKC; kp += 2) {
      float2 av[C::TM], bv[C::TN];
#pragma unroll
      for (int x = 0; x < C::TM; ++x) av[x] = As[(arow0 + 32 * x) * C::LDA + kp + h];
#pragma unroll
      for (int y = 0; y < C::TN; ++y) bv[y] = Bs[(bcol0 + C::CPT * y) * C::LDA + kp + h];
      if constexpr (G3) {
        float as[C::TM];
#pragma unroll
        for (int x = 0; x < C::TM; ++x) as[x] = av[x].x + av[x].y;
#pragma unroll
        for (int y = 0; y < C::TN; ++y) {
          const float bs = bv[y].x + bv[y].y;
#pragma unroll
          for (int x = 0; x < C::TM; ++x) {
            acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[x].x, bv[y].x, acc[x][y], 0, 0, 0);
            acc2[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[x].y, bv[y].y, acc2[x][y], 0, 0, 0);
            acc3[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(as[x], bs, acc3[x][y], 0, 0, 0);
          }
        }
      } else {
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
  }

  // epilogue: pdep is additive over disjoint bit groups of the row index
  // (split-K partials: plain row-major, the row bits above the column bits)
  const uint64_t maskA = SPLITK ? ((uint64_t)(M - 1) << d.n) : d.cmask;
  const uint64_t maskB = ~maskA & ((1ull << (d.m + d.n)) - 1);
  const uint64_t row_base = (uint64_t)(bm * BM + wm * C::WM + 4 * h);
  const uint64_t pbase = pdep64(row_base, maskA);
  uint64_t pq[4], pg[4], pt[C::TM];
#pragma unroll
  for (int q = 0; q < 4; ++q) pq[q] = pdep64((uint64_t)q, maskA);
#pragma unroll
  for (int g = 0; g < 4; ++g) pg[g] = pdep64((uint64_t)(8 * g), maskA);
#pragma unroll
  for (int x = 0; x < C::TM; ++x) pt[x] = pdep64((uint64_t)(32 * x), maskA);
  // the output's two lowest bits are row bits 0 and 1: a lane's four
  // accumulators q = 0..3 are four consecutive outputs (16-byte stores)
  const bool rows4 = (maskA & 3) == 3;
  float vmax = 0.f;
#pragma unroll
  for (int y = 0; y < C::TN; ++y) {
    uint64_t ncol = (uint64_t)(bn * BNC + bcol0 + C::CPT * y);
    uint64_t pn = pdep64(ncol, maskB);
#pragma unroll
    for (int x = 0; x < C::TM; ++x)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        if constexpr (G3) {
          // whole complex outputs: Re = P1 - P2, Im = P3 - P1 - P2
          float vr[4], vi[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float p1 = acc[x][y][4 * g + q], p2 = acc2[x][y][4 * g + q];
            vr[q] = p1 - p2;
            vi[q] = acc3[x][y][4 * g + q] - p1 - p2;
            vmax = fmaxf(vmax, fmaxf(fabsf(vr[q]), fabsf(vi[q])));
          }
          if (rows4) {
            const uint64_t a0 = pbase | pt[x] | pg[g] | pn;
            if (!SPLITK && d.split_out) {
              // one split group: 16 bytes of hi words, then 16 bytes of lo words
              uint32_t hw[4], lw[4];
#pragma unroll
              for (int q = 0; q < 4; ++q)
                hw[q] = d.split_out == 1 ? split_pair<true>(vr[q], vi[q], 1.f, lw[q])
                                         : split_pair<false>(vr[q], vi[q], so, lw[q]);
              uint4* g4 = reinterpret_cast<uint4*>(Cw) + (a0 >> 2) * 2;
              g4[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
              g4[1] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
            } else {
              float4* c4 = reinterpret_cast<float4*>(Cf + 2 * a0);
              c4[0] = make_float4(vr[0], vi[0], vr[1], vi[1]);
              c4[1] = make_float4(vr[2], vi[2], vr[3], vi[3]);
            }
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const uint64_t addr = pbase | pt[x] | pg[g] | pq[q] | pn;
              if (!SPLITK && d.split_out == 1)
                store_split<true>(Cw, addr, vr[q], vi[q], 1.f);
              else if (!SPLITK && d.split_out)
                store_split<false>(Cw, addr, vr[q], vi[q], so);
              else
                reinterpret_cast<float2*>(Cf)[addr] = make_float2(vr[q], vi[q]);
            }
          }
          continue;
        }
        if (rows4) {
          const uint64_t a0 = pbase | pt[x] | pg[g] | pn;
          float v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            v[q] = acc[x][y][4 * g + q];
            vmax = fmaxf(vmax, fabsf(v[q]));
          }
          if (!SPLITK && d.split_out) {
            // the even lane writes the four hi words, the odd lane the lo words
            uint32_t wd[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float o = __shfl_xor(v[q], 1, 64);
              const float re = im_col ? o : v[q], im = im_col ? v[q] : o;
              uint32_t lo, hi;
              if (d.split_out == 1)
                hi = split_pair<true>(re, im, 1.f, lo);
              else
                hi = split_pair<false>(re, im, so, lo);
              wd[q] = im_col ? lo : hi;
            }
            *reinterpret_cast<uint4*>(Cw + (a0 >> 2) * 8 + (im_col ? 4 : 0)) =
                make_uint4(wd[0], wd[1], wd[2], wd[3]);
          } else {
            // even lane (re parts): outputs 0, 1; odd lane (im parts): outputs 2, 3
            const float s0 = __shfl_xor(im_col ? v[0] : v[2], 1, 64);
            const float s1 = __shfl_xor(im_col ? v[1] : v[3], 1, 64);
            *reinterpret_cast<float4*>(Cf + 2 * a0 + (im_col ? 4 : 0)) =
                im_col ? make_float4(s0, v[2], s1, v[3]) : make_float4(v[0], s0, v[1], s1);
          }
          continue;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint64_t addr = pbase | pt[x] | pg[g] | pq[q] | pn;
          float v = acc[x][y][4 * g + q];
          vmax = fmaxf(vmax, fabsf(v));
          if (!SPLITK && d.split_out) {
            // re and im of this output sit on neighbouring lanes: the even
            // lane writes the hi word, the odd lane the lo word
            const float o = __shfl_xor(v, 1, 64);
            const float re = im_col ? o : v, im = im_col ? v : o;
            uint32_t lo, hi;
            if (d.split_out == 1)
              hi = split_pair<true>(re, im, 1.f, lo);
            else
              hi = split_pair<false>(re, im, so, lo);
            Cw[(addr >> 2) * 8 + (im_col ? 4 : 0) + (addr & 3)] = im_col ? lo : hi;
          } else {
            Cf[2 * addr + (im_col ? 1 : 0)] = v;
          }
        }
      }
  }
  if (!SPLITK && d.scale_c) record_max(d.scale_c + b, vmax);
}

// Second pass of the split-K GEMM: C[b][merge(row, column)] = the chunks'
// partials added in FP32 in chunk order. One thread per output; 2^(m+n) is
// a multiple of the block size, so a block (and a wave) stays in one slice.
__global__ __launch_bounds__(256) void k_splitk_reduce(GemmDesc d) {
  const int64_t MN = int64_t(1) << (d.m + d.n);
  const int chunks = 1 << (d.k - d.kc_bits);
  const uint64_t full = (1ull << (d.m + d.n)) - 1;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t b = i >> (d.m + d.n), e = i & (MN - 1);
  const float2* src = d.part + (b * chunks) * MN + e;
  float re = 0.f, im = 0.f;
  for (int c = 0; c < chunks; ++c) {
    const float2 v = src[c * MN];
    re += v.x;
    im += v.y;
  }
  const uint64_t row = (uint64_t)e >> d.n, col = (uint64_t)e & ((1ull << d.n) - 1);
  d.C[b * d.sC + (pdep64(row, d.cmask) | pdep64(col, ~d.cmask & full))] = make_float2(re, im);
  if (d.scale_c) record_max(d.scale_c + b, fmaxf(fabsf(re), fabsf(im)));
}


template <bool BF>
__device__ __forceinline__ floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c) {
  if constexpr (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(typename SplitType<true>::V8, a),
                                                   __builtin_bit_cast(typename SplitType<true>::V8, b),
                                                   c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(typename SplitType<false>::V8, a),
                                                  __builtin_bit_cast(typename SplitType<false>::V8, b),
                                                  c, 0, 0, 0);
}

// B operand of output real parts: (re, -im) pairs; imaginary parts: (im, re)
// (whole-vector operations: element-wise bit casts of vector elements were
// miscompiled by this toolchain)
__device__ __forceinline__ u32x4 bform(u32x4 w, bool im_col) {
  if (im_col) return (w << 16) | (w >> 16);
  return w ^ 0x80000000u;
}

// hi * 2^11 for eight packed fp16 values (exact: a power-of-two scaling)
__device__ __forceinline__ u32x4 times2048(u32x4 w) {
  typedef _Float16 H8 __attribute__((ext_vector_type(8)));
  H8 h = __builtin_bit_cast(H8, w);
  h = h * (_Float16)2048.0f;
  return __builtin_bit_cast(u32x4, h);
}

// complex64 -> split layout of one tensor for nb slices (src and dst may
// be the same buffer).
template <bool BF>
__global__ __launch_bounds__(256) void k_split_convert(const float2* X, float2* Y, int64_t per_slice,
                                                       int nb, const uint32_t* slot) {
  const int64_t groups = per_slice / 4;
  const int64_t total = groups * nb;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    int64_t b = g / groups;
    float sigma = BF ? 1.f : scale_of(slot[b]);
    const float4* p = reinterpret_cast<const float4*>(X) + 2 * g;
    float4 u = p[0], v = p[1];
    uint4 hi, lo;
    hi.x = split_pair<BF>(u.x, u.y, sigma, lo.x);
    hi.y = split_pair<BF>(u.z, u.w, sigma, lo.y);
    hi.z = split_pair<BF>(v.x, v.y, sigma, lo.z);
    hi.w = split_pair<BF>(v.z, v.w, sigma, lo.w);
    uint4* q = reinterpret_cast<uint4*>(Y) + 2 * g;
    q[0] = hi;
    q[1] = lo;
  }
}

// Split GEMM tile: NWM x NWN waves, wave tile (BM/NWM) rows x (BNC/NWN)
// complex columns. MFMA columns are complex outputs: each lane reads its B
// value once and forms both real-form rows of it, (re, -im) for the real
// accumulator and (im, re) for the imaginary one; the forms of one B
// fragment feed the wave's TM row tiles.
template <int BM, int BNC, int BKC, int NWN, int NWM = 2>
struct SplitCfg {
  static constexpr int WM = BM / NWM, TM = WM / 32;
  static constexpr int WNC = BNC / NWN, TN = WNC / 32;
  static_assert(TM >= 1 && TN >= 1 && BKC % 8 == 0, "tile too small for the split GEMM");
};

// Two or three waves per SIMD where the registers allow it without spilling (the
// accumulators then live in VGPRs), so that one block's LDS staging and
// barriers overlap another block's matrix work.
//
// Two ways of staging the operand tiles in LDS (DMA template flag):
//  * through registers: each k-tile is loaded into registers while the
//    previous one is computed, then written to LDS between two barriers;
//    LDS rows are padded (row r starts at unit U r + r / (16 / U));
//  * DMA: global_load_lds writes each wave's 64 x 16 bytes straight into
//    LDS (lane i to unit i of the destination), two LDS stages, one barrier
//    per k-tile, no staging registers. Each lane picks its global chunk so
//    that unit U r + (g ^ sw(r)) of a part array holds group g of row r,
//    sw(r) = (r / (16 / U)) mod U: 16 consecutive rows at one group then fall
//    on 16 distinct units (all 64 banks) as with the padding.
//
// NWM x NWN waves per block: 2 x 2 as a rule; 2 x 4 with DMA staging puts
// four waves on each SIMD (two blocks of eight) to hide LDS and barrier
// latency behind more independent matrix work; wave tiles of four row tiles
// (1 x 4 waves on 128 x 128, 2 x 2 on 256 x 64) halve the operand-form
// work per matrix instruction.
template <int BM, int BNC, int BKC, bool BF, bool DMA, int NWN = 2, int NWM = 2>
__global__ __launch_bounds__(64 * NWM * NWN, NWM * NWN == 8 ? 2 : ((BM * BNC >= 16384 && BKC >= 32) ? 1 : (BM * BNC >= 16384 || BKC >= 32 ? 2 : 3))) void k_cgemm_split(GemmDesc d) {
  static_assert((NWN == 2 && NWM == 2) || DMA, "other wave layouts need DMA staging");
  constexpr int NW = NWM * NWN;  // waves per block
  using C = SplitCfg<BM, BNC, BKC, NWN, NWM>;
  // LDS rows of U 16-byte units (one unit = 4 complex of hi or lo parts);
  // row r starts at unit U r + r / (16 / U), so that 16 consecutive rows at
  // one group (a read pass) and the 16 / U rows x U groups of a store pass
  // each fall on 16 distinct units, i.e. on all 64 banks once
  constexpr int U = BKC / 4;
  constexpr int RPP = 16 / U;               // rows per 16-chunk store pass
  constexpr int CHA = BM * U * 2;           // 16-byte chunks (hi and lo)
  constexpr int CHB = BNC * U * 2;
  constexpr int RA = (CHA + 255) / 256, RB = (CHB + 255) / 256;
  static_assert(BM % RPP == 0 && BNC % RPP == 0, "tile rows must fill store passes");
  constexpr int SA = BM * U, SB = BNC * U;  // DMA: units per part array and stage
  static_assert(!DMA || (SA % 64 == 0 && SB % 64 == 0 && ((SA + SB) / 32) % NW == 0),
                "DMA staging needs whole 64-unit slots, a multiple of the wave count per stage");
  __shared__ u32x4 Ahi[DMA ? 1 : BM * U + BM / RPP], Alo[DMA ? 1 : BM * U + BM / RPP];
  __shared__ u32x4 Bhi[DMA ? 1 : BNC * U + BNC / RPP], Blo[DMA ? 1 : BNC * U + BNC / RPP];
  // DMA stages: [stage][Ahi SA | Alo SA | Bhi SB | Blo SB]
  constexpr int STG = 2 * (SA + SB);
  __shared__ u32x4 Sd[DMA ? 2 * STG : 1];
  auto unit = [](int row, int g) {
    if constexpr (DMA)
      return U * row + (g ^ ((row / RPP) % U));
    else
      return U * row + row / RPP + g;
  };

  const int64_t M = int64_t(1) << d.m, N = int64_t(1) << d.n, K = int64_t(1) << d.k;
  int64_t b, bm, bn;
  tile_of(blockIdx.x, M / BM, N / BNC, d.nb, b, bm, bn);

  const float sa = BF ? 1.f : scale_of(d.scale_a[b]), sb = BF ? 1.f : scale_of(d.scale_b[b]);
  const float so = !BF && d.split_out ? split_out_scale(d, b, K, bm == 0 && bn == 0 && threadIdx.x == 0) : 1.f;
  // operands in split layout: a row of K complex is K / 4 groups of 32 bytes
  const u32x4* A = reinterpret_cast<const u32x4*>(d.A + b * d.sA + bm * BM * K);
  const u32x4* B = reinterpret_cast<const u32x4*>(d.B + b * d.sB + bn * BNC * K);
  float2* Cc = d.C + b * d.sC;

  // the wave index is uniform: keep it scalar so that per-wave choices branch on SGPRs
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / NWN, wn = wave % NWN;
  const int h = lane >> 5, i = lane & 31;

  floatx16 are[C::TM][C::TN], aim[C::TM][C::TN];
#pragma unroll
  for (int x = 0; x < C::TM; ++x)
#pragma unroll
    for (int y = 0; y < C::TN; ++y)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        are[x][y][v] = 0.f;
        aim[x][y][v] = 0.f;
      }

  // chunk c: 32 consecutive chunks cover RPP rows x U groups, first the
  // 16 hi parts then the 16 lo parts (hi and lo of a group are adjacent in
  // memory, so a row's cache line is read by one instruction)
  auto chunk = [](int c, int& row, int& g, int& lo) {
    int j = c & 15;
    lo = (c >> 4) & 1;
    row = (c >> 5) * RPP + j / U;
    g = j % U;
  };
  u32x4 ra[RA], rb[RB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int c = tid + 256 * r;
      if (c < CHA) {
        int row, g, lo;
        chunk(c, row, g, lo);
        ra[r] = A[(row * K + k0) / 2 + 2 * g + lo];
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int c = tid + 256 * r;
      if (c < CHB) {
        int row, g, lo;
        chunk(c, row, g, lo);
        rb[r] = B[(row * K + k0) / 2 + 2 * g + lo];
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      int c = tid + 256 * r;
      if (c < CHA) {
        int row, g, lo;
        chunk(c, row, g, lo);
        if (lo)
          Alo[unit(row, g)] = ra[r];
        else
          Ahi[unit(row, g)] = ra[r];
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int c = tid + 256 * r;
      if (c < CHB) {
        int row, g, lo;
        chunk(c, row, g, lo);
        if (lo)
          Blo[unit(row, g)] = rb[r];
        else
          Bhi[unit(row, g)] = rb[r];
      }
    }
  };

  const int arow0 = wm * C::WM + i;
  const int bcol0 = wn * C::WNC + i;

  // DMA: slot t (64 units) of a stage -> part array and offset; lane i
  // fetches the chunk that belongs at unit 64 q + i of that array
  auto dma = [&](int stage, int64_t k0) {
    constexpr int T = STG / 64;
#pragma unroll
    for (int j = 0; j < T / NW; ++j) {
      const int t = wave + NW * j;
      const int tA = SA / 64, tB = SB / 64;
      int q, lo;
      const u32x4* src;
      int base;
      if (t < 2 * tA) {
        lo = t >= tA;
        q = t - lo * tA;
        src = A;
        base = lo * SA;
      } else {
        const int tb = t - 2 * tA;
        lo = tb >= tB;
        q = tb - lo * tB;
        src = B;
        base = 2 * SA + lo * SB;
      }
      const int pu = 64 * q + lane;
      const int row = pu / U, g = (pu % U) ^ ((row / RPP) % U);
      __builtin_amdgcn_global_load_lds(
          (const void*)(src + ((int64_t)row * (K >> 1) + (k0 >> 1) + 2 * g + lo)),
          (__attribute__((address_space(3))) void*)(Sd + stage * STG + base + 64 * q), 16, 0, 0);
    }
  };

  if constexpr (DMA) dma(0, 0); else load(0);
  for (int64_t k0 = 0; k0 < K; k0 += BKC) {
    const u32x4 *SAh, *SAl, *SBh, *SBl;
    if constexpr (DMA) {
      const int stage = (int)((k0 / BKC) & 1);
      __builtin_amdgcn_s_waitcnt(0);  // this wave's copies into the stage have landed
      __syncthreads();                // everyone's have, and the other stage is free
      if (k0 + BKC < K) dma(stage ^ 1, k0 + BKC);
      SAh = Sd + stage * STG;
      SAl = SAh + SA;
      SBh = SAh + 2 * SA;
      SBl = SBh + SB;
    } else {
      __syncthreads();
      stash();
      __syncthreads();
      if (k0 + BKC < K) load(k0 + BKC);
      SAh = Ahi;
      SAl = Alo;
      SBh = Bhi;
      SBl = Blo;
    }
#pragma unroll
    for (int ch = 0; ch < BKC / 8; ++ch) {
      const int gl = 2 * ch + h;  // this lane's group: 8 k' = 4 complex
      u32x4 ah[C::TM], al[C::TM];
#pragma unroll
      for (int x = 0; x < C::TM; ++x) {
        int o = unit(arow0 + 32 * x, gl);
        ah[x] = SAh[o];
        al[x] = SAl[o];
      }
#pragma unroll
      for (int y = 0; y < C::TN; ++y) {
        int o = unit(bcol0 + 32 * y, gl);
        u32x4 bh = SBh[o];
        u32x4 bl = SBl[o];
        u32x4 bs = BF ? bh : times2048(bh);
        u32x4 rh = bform(bh, false), ih = bform(bh, true);
        u32x4 rl = bform(bl, false), il = bform(bl, true);
        u32x4 rs = BF ? rh : bform(bs, false), is = BF ? ih : bform(bs, true);
#pragma unroll
        for (int x = 0; x < C::TM; ++x) {
          are[x][y] = mfma16<BF>(ah[x], rs, are[x][y]);
          are[x][y] = mfma16<BF>(ah[x], rl, are[x][y]);
          are[x][y] = mfma16<BF>(al[x], rh, are[x][y]);
          aim[x][y] = mfma16<BF>(ah[x], is, aim[x][y]);
          aim[x][y] = mfma16<BF>(ah[x], il, aim[x][y]);
          aim[x][y] = mfma16<BF>(al[x], ih, aim[x][y]);
        }
      }
    }
  }

  const float post = BF ? 1.f : (1.0f / 2048.0f) / sa / sb;
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
  // the output's two lowest bits are row bits 0 and 1: a lane's four
  // accumulators q = 0..3 are four consecutive outputs (16-byte stores)
  const bool rows4 = (maskA & 3) == 3;
  float vmax = 0.f;
#pragma unroll
  for (int y = 0; y < C::TN; ++y) {
    uint64_t pn = pdep64((uint64_t)(bn * BNC + bcol0 + 32 * y), maskB);
#pragma unroll
    for (int x = 0; x < C::TM; ++x)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        if (rows4) {
          const uint64_t a0 = pbase | pt[x] | pg[g] | pn;
          float vr[4], vi[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            vr[q] = are[x][y][4 * g + q] * post;
            vi[q] = aim[x][y][4 * g + q] * post;
            vmax = fmaxf(vmax, fmaxf(fabsf(vr[q]), fabsf(vi[q])));
          }
          if (d.split_out) {
            // one split group: 16 bytes of hi words, then 16 bytes of lo words
            uint32_t hw[4], lw[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) hw[q] = split_pair<BF>(vr[q], vi[q], so, lw[q]);
            uint4* g4 = reinterpret_cast<uint4*>(Cc) + (a0 >> 2) * 2;
            g4[0] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
            g4[1] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
          } else {
            float4* c4 = reinterpret_cast<float4*>(Cc + a0);
            c4[0] = make_float4(vr[0], vi[0], vr[1], vi[1]);
            c4[1] = make_float4(vr[2], vi[2], vr[3], vi[3]);
          }
          continue;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint64_t addr = pbase | pt[x] | pg[g] | pq[q] | pn;
          float vr = are[x][y][4 * g + q] * post, vi = aim[x][y][4 * g + q] * post;
          vmax = fmaxf(vmax, fmaxf(fabsf(vr), fabsf(vi)));
          if (d.split_out)
            store_split<BF>(reinterpret_cast<uint32_t*>(Cc), addr, vr, vi, so);
          else
            Cc[addr] = make_float2(vr, vi);
        }
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
    // three real products per complex product (configurations 10-15)
    {128, 64, 16, "c64_3m_128x64x16"}, {128, 128, 16, "c64_3m_128x128x16"},
    {256, 64, 16, "c64_3m_256x64x16"}, {64, 64, 16, "c64_3m_64x64x16"},
    {128, 64, 32, "c64_3m_128x64x32"}, {128, 32, 16, "c64_3m_128x32x16"},
};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
const CfgInfo kSplitCfgs[] = {
    {128, 128, 16, "split_128x128x16"}, {128, 64, 16, "split_128x64x16"}, {64, 128, 16, "split_64x128x16"},
    {64, 64, 16, "split_64x64x16"},     {128, 64, 32, "split_128x64x32"}, {128, 64, 64, "split_128x64x64"},
    {64, 64, 8, "split_64x64x8"},       {128, 128, 32, "split_128x128x32"}, {64, 64, 32, "split_64x64x32"},
    {64, 128, 32, "split_64x128x32"},
    // operand tiles staged by global_load_lds, two LDS stages
    {128, 128, 16, "split_dma_128x128x16"}, {128, 64, 16, "split_dma_128x64x16"},
    {64, 128, 16, "split_dma_64x128x16"},   {64, 64, 16, "split_dma_64x64x16"},
    {64, 64, 8, "split_dma_64x64x8"},
    // eight waves per block (2 x 4), DMA staging
    {128, 128, 16, "split_dma8w_128x128x16"},
    // wave tiles of 128 rows x 32 complex columns (DMA staging)
    {128, 128, 16, "split_dma1x4_128x128x16"}, {256, 64, 16, "split_dma2x2_256x64x16"},
};
constexpr int kNumSplit = sizeof(kSplitCfgs) / sizeof(kSplitCfgs[0]);

template <int BM, int BNC, int BKC, int NWN = 2, bool G3 = false, int MINW = 1>
void run(const GemmDesc& d, hipStream_t st) {
  int64_t tiles = ((int64_t(1) << d.m) / BM) * ((int64_t(1) << d.n) / BNC) * d.nb;
  hipLaunchKernelGGL((k_cgemm_c64<BM, BNC, BKC, NWN, false, G3, MINW>), dim3((unsigned)tiles), dim3(256), 0, st, d);
}

// Split-K tiles: waves 4 x 1 for 16 and 32 complex columns, 2 x 2 otherwise;
// configurations 4, 5 and 7 take the three-product form; 6 and 7 fit
// products with 64 rows (the gradient's adjoint products).
struct SplitKCfg {
  int bm, bnc, bkc;
  const char* name;
};
const SplitKCfg kSplitKCfgs[] = {
    {128, 16, 16, "splitk_128x16x16"},
    {256, 16, 16, "splitk_256x16x16"},
    {128, 32, 16, "splitk_128x32x16"},
    {128, 64, 16, "splitk_128x64x16"},
    {128, 64, 16, "splitk_3m_128x64x16"},
    {128, 32, 16, "splitk_3m_128x32x16"},
    {64, 32, 16, "splitk_64x32x16"},
    {64, 64, 16, "splitk_3m_64x64x16"},
};
constexpr int kNumSplitK = sizeof(kSplitKCfgs) / sizeof(kSplitKCfgs[0]);

template <int BM, int BNC, int BKC, int NWN, bool G3 = false, int MINW = 1>
void run_splitk(const GemmDesc& d, hipStream_t st) {
  const int64_t chunks = int64_t(1) << (d.k - d.kc_bits);
  const int64_t blocks = ((int64_t(1) << d.m) / BM) * ((int64_t(1) << d.n) / BNC) * d.nb * chunks;
  hipLaunchKernelGGL((k_cgemm_c64<BM, BNC, BKC, NWN, true, G3, MINW>), dim3((unsigned)blocks), dim3(256), 0, st, d);
  const int64_t outs = (int64_t(1) << (d.m + d.n)) * d.nb;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)(outs / 256)), dim3(256), 0, st, d);
}

template <int BM, int BNC, int BKC, bool DMA = false, int NWN = 2, int NWM = 2>
void run_split(const GemmDesc& d, bool bf, hipStream_t st) {
  int64_t tiles = ((int64_t(1) << d.m) / BM) * ((int64_t(1) << d.n) / BNC) * d.nb;
  const dim3 block(64 * NWM * NWN);
  if (bf)
    hipLaunchKernelGGL((k_cgemm_split<BM, BNC, BKC, true, DMA, NWN, NWM>), dim3((unsigned)tiles), block, 0, st, d);
  else
    hipLaunchKernelGGL((k_cgemm_split<BM, BNC, BKC, false, DMA, NWN, NWM>), dim3((unsigned)tiles), block, 0, st, d);
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

// About 2^12 (tile, chunk) pairs per slice for a 128 x 16 tile, each chunk
// at least 2^8 long; offered only for sums of 2^10 and more.
int splitk_chunk_bits(int m, int k, int n) {
  if (k < 10 || m >= 40 || n >= 40) return 0;
  int c = 23 - (m + n);
  if (c > k - 8) c = k - 8;
  return c > 0 ? c : 0;
}

int splitk_config_count() { return kNumSplitK; }

bool splitk_config_fits(int cfg, int m, int k, int n) {
  if (cfg < 0 || cfg >= kNumSplitK) return false;
  const int c = splitk_chunk_bits(m, k, n);
  const SplitKCfg& t = kSplitKCfgs[cfg];
  return c > 0 && (1ll << m) >= t.bm && (1ll << n) >= t.bnc && (1ll << (k - c)) >= t.bkc;
}

const char* splitk_config_name(int cfg) { return cfg >= 0 && cfg < kNumSplitK ? kSplitKCfgs[cfg].name : "?"; }

int64_t splitk_part_elems(int m, int k, int n) {
  for (int c = 0; c < kNumSplitK; ++c)
    if (splitk_config_fits(c, m, k, n) || splitk_config_fits(c, n, k, m))
      return (int64_t(1) << splitk_chunk_bits(m, k, n)) << (m + n);
  return 0;
}

void launch_cgemm_splitk(const GemmDesc& d0, hipStream_t st) {
  GemmDesc d = d0;
  d.kc_bits = d.k - splitk_chunk_bits(d.m, d.k, d.n);
  switch (d.cfg) {
    case 0: run_splitk<128, 16, 16, 1>(d, st); break;
    case 1: run_splitk<256, 16, 16, 1>(d, st); break;
    case 2: run_splitk<128, 32, 16, 1>(d, st); break;
    case 3: run_splitk<128, 64, 16, 2>(d, st); break;
    case 4: run_splitk<128, 64, 16, 2, true, 3>(d, st); break;
    case 5: run_splitk<128, 32, 16, 1, true>(d, st); break;
    case 6: run_splitk<64, 32, 16, 2>(d, st); break;
    case 7: run_splitk<64, 64, 16, 2, true>(d, st); break;
  }
}

void launch_split_convert(const float2* X, float2* Y, int rank, int nb, const uint32_t* slot,
                          int mode, hipStream_t st) {
  int64_t per = int64_t(1) << rank;
  int64_t groups = per / 4 * nb;
  int64_t blocks = (groups + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (mode == LTN_SPLIT_BF16)
    hipLaunchKernelGGL(k_split_convert<true>, dim3((unsigned)blocks), dim3(256), 0, st, X, Y, per, nb,
                       slot);
  else
    hipLaunchKernelGGL(k_split_convert<false>, dim3((unsigned)blocks), dim3(256), 0, st, X, Y, per, nb,
                       slot);
}

void launch_cgemm(const GemmDesc& d, int mode, hipStream_t st) {
  if (mode != LTN_C64) {
    bool bf = mode == LTN_SPLIT_BF16;
    switch (d.cfg) {
      case 0: run_split<128, 128, 16>(d, bf, st); break;
      case 1: run_split<128, 64, 16>(d, bf, st); break;
      case 2: run_split<64, 128, 16>(d, bf, st); break;
      case 3: run_split<64, 64, 16>(d, bf, st); break;
      case 4: run_split<128, 64, 32>(d, bf, st); break;
      case 5: run_split<128, 64, 64>(d, bf, st); break;
      case 6: run_split<64, 64, 8>(d, bf, st); break;
      case 7: run_split<128, 128, 32>(d, bf, st); break;
      case 8: run_split<64, 64, 32>(d, bf, st); break;
      case 9: run_split<64, 128, 32>(d, bf, st); break;
      case 10: run_split<128, 128, 16, true>(d, bf, st); break;
      case 11: run_split<128, 64, 16, true>(d, bf, st); break;
      case 12: run_split<64, 128, 16, true>(d, bf, st); break;
      case 13: run_split<64, 64, 16, true>(d, bf, st); break;
      case 14: run_split<64, 64, 8, true>(d, bf, st); break;
      case 15: run_split<128, 128, 16, true, 4>(d, bf, st); break;
      case 16: run_split<128, 128, 16, true, 4, 1>(d, bf, st); break;
      case 17: run_split<256, 64, 16, true, 2, 2>(d, bf, st); break;
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
    case 10: run<128, 64, 16, 2, true, 3>(d, st); break;
    case 11: run<128, 128, 16, 2, true>(d, st); break;
    case 12: run<256, 64, 16, 2, true>(d, st); break;
    case 13: run<64, 64, 16, 2, true>(d, st); break;
    case 14: run<128, 64, 32, 2, true>(d, st); break;
    case 15: run<128, 32, 16, 1, true>(d, st); break;
  }
}

}  // namespace ltn
