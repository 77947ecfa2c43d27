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
          Cf[2 * addr + (im_col ? 1 : 0)] = acc[x][y][4 * g + q];
        }
  }
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

template <int BM, int BNC, int BKC>
void run(const GemmDesc& d, hipStream_t st) {
  int64_t tiles = ((int64_t(1) << d.m) / BM) * ((int64_t(1) << d.n) / BNC) * d.nb;
  hipLaunchKernelGGL((k_cgemm_c64<BM, BNC, BKC>), dim3((unsigned)tiles), dim3(256), 0, st, d);
}

}  // namespace

int gemm_config_count() { return kNumCfgs; }

bool gemm_config_fits(int cfg, int m, int k, int n) {
  if (cfg < 0 || cfg >= kNumCfgs) return false;
  const CfgInfo& c = kCfgs[cfg];
  return m < 40 && n < 40 && (1ll << m) >= c.bm && (1ll << n) >= c.bnc && (1ll << k) >= c.bkc;
}

const char* gemm_config_name(int cfg) { return cfg >= 0 && cfg < kNumCfgs ? kCfgs[cfg].name : "?"; }

void launch_cgemm(const GemmDesc& d, int mode, hipStream_t st) {
  (void)mode;
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
