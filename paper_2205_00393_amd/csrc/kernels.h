// Device kernels of libltn and their host-side launchers (all asynchronous
// on the given stream). Tensors are complex64 (float2); each batched
// operand is a base pointer plus a per-slice stride in elements.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "ltn.h"

namespace ltn {

// Raise a per-slice maximum slot (bits of a non-negative float) to v. The
// slot only grows, so when a plain read already shows at least v the
// atomic is skipped (a stale read can only cost an extra atomic); this
// keeps thousands of tiles from serialising on one address.
__device__ __forceinline__ void raise_max(uint32_t* slot, float v) {
  const uint32_t bits = __float_as_uint(v);
  if (v > 0.f && *reinterpret_cast<volatile uint32_t*>(slot) < bits) atomicMax(slot, bits);
}

constexpr int kMaxLeafRank = 32;

// Gather of one leaf into its per-slice layout (Sec. 2.1.1: a sliced index
// takes the value given by the slice id).
// leaf gather: elements per block (a leaf of 2^rank elements takes
// ceil(2^rank / kGatherChunk) blocks per slice)
constexpr int64_t kGatherChunk = 4096;

struct GatherDesc {
  int64_t src_off;   // element offset in the leaf-data area
  int64_t chunk0;    // first block (chunk) of this leaf in the flattened gather grid
  int64_t tensor;    // tensor id (slot of its per-slice max in split modes)
  int64_t dst_off;   // element offset of slice 0 in the arena
  int32_t rank;      // unsliced rank (dst has 2^rank elements per slice)
  int32_t nsl;       // number of sliced axes
  int8_t src_bit[kMaxLeafRank];
  int8_t sl_src_bit[kMaxLeafRank];
  int8_t sl_bit[kMaxLeafRank];
};

struct ParamLeaf {
  int64_t src_off;   // element offset of the 2x2 [out][in] data
  int32_t gate;      // u3 gate number (angles 3*gate .. 3*gate+2)
  int32_t gd;        // index of its GatherDesc (for cotangent scatter)
};

// Operand addressing of the generic contraction
//   out[pdep(x, ox) | pdep(y, oy)] = sum_z P[pdep(x, px) | pdep(z, pz)]
//                                        * Q[pdep(y, qy) | pdep(z, qz)]
struct GenericDesc {
  const float2* P;
  const float2* Q;
  float2* out;
  int64_t sP, sQ, sO;    // per-slice strides (elements)
  uint64_t px, pz, qy, qz, ox, oy;
  int32_t xb, yb, zb;    // bit counts
  int32_t conjQ;
  int32_t accumulate;    // add into out instead of overwrite
  int32_t nb;            // slices
  uint32_t* scale_out;   // if set: record the output's per-slice max |x|
};

void launch_set_ids(uint64_t* d_ids, const uint64_t* h_ids, int n, hipStream_t st);
void launch_set_range(uint64_t* d_ids, uint64_t base, int n, hipStream_t st);
void launch_gather(const GatherDesc* d_desc, int n_leaves, int64_t n_chunks, int max_elems,
                   const float2* leafdata, float2* arena, const uint64_t* ids, int nb, uint32_t* scales,
                   int bstride, hipStream_t st);
void launch_reduce(const float2* root, int rank, uint64_t out_mask, const int32_t* sl_bits,
                   const int32_t* out_bits, int n_sl, const uint64_t* ids, int nb, double* out,
                   hipStream_t st);
void launch_root_cotangent(const double* cot, int rank, uint64_t out_mask, const int32_t* sl_bits,
                           const int32_t* out_bits, int n_sl, const uint64_t* ids, int nb,
                           float2* rootcot, hipStream_t st);
void launch_u3_build(const ParamLeaf* d_pl, int n, const double* angles, float2* leafdata,
                     hipStream_t st);
void launch_leaf_cot_accumulate(const ParamLeaf* d_pl, int n, const GatherDesc* gd,
                                const float2* cot_arena, const uint64_t* ids, int nb,
                                double* leafgrad, hipStream_t st);
void launch_u3_adjoint(const ParamLeaf* d_pl, int n, const double* angles, const double* leafgrad,
                       double* angle_grad, hipStream_t st);
void launch_fill_zero(void* p, size_t bytes, hipStream_t st);
void launch_generic(const GenericDesc& d, int tk, hipStream_t st);
// n independent descriptors (device array) in one launch over nb slices;
// max_outs: largest 2^(xb + yb) among them
void launch_generic_multi(const GenericDesc* d_descs, int n, uint64_t max_outs, int nb, int tk,
                          hipStream_t st);

// C[merge(m, n)] = sum_k A[m 2^k + k] B[n 2^k + k] on FP32 MFMA; the output
// bit j comes from A's next free bit if (cmask >> j) & 1, else from B's.
struct GemmDesc {
  const float2* A;
  const float2* B;
  float2* C;
  int64_t sA, sB, sC;
  int32_t m, k, n;
  uint64_t cmask;
  int32_t nb;
  int32_t cfg;             // tile configuration id (per mode)
  const uint32_t* scale_a;   // split modes: per-slice max |x| (float bits) of A
  const uint32_t* scale_b;   //              and of B
  uint32_t* scale_c;         // if set: record the output's per-slice max |x|
  int32_t split_out;         // write C in the split layout: 0 no, 1 bf16, 2 fp16
  const uint32_t* max_a;     // split_out 2: recorded max |Re|, |Im| of A and of B,
  const uint32_t* max_b;     //   whose bound 2 K max_a max_b sets C's fp16 scale
  uint32_t* bound_c;         //   and is stored here per slice for the consumer
  float2* part;              // split-K: [nb][chunks][2^(m+n)] FP32 partial sums
  int32_t kc_bits;           // split-K: log2 of the sum length of one chunk
};
// Tile plan of a bit permutation (built on the host by ltn_permute).
struct PermuteDesc {
  int32_t rank, n_tile, n_outer;
  int64_t batch;
  uint64_t flip;         // XORed into every element (1 << 63: complex conjugate)
  int8_t tile_src[16];   // tile bit k -> source bit (ascending)
  int8_t tile_dst[16];   // destination-order rank r -> destination bit
  int8_t dst_tile[16];   // destination-order rank r -> tile bit
  int8_t outer_src[64];  // outer bit k -> source bit
  int8_t outer_dst[64];  // outer bit k -> destination bit
  uint8_t swz[8];        // tile bit 5 + k -> XOR mask on the low 5 bits of its LDS slot
};
void launch_permute(const float2* in, float2* out, const PermuteDesc& d, hipStream_t st);

// Narrow step C[merge(m, n)] = sum_k A[m][k] B[n][k] (k + n <= 10, n <= 6), A and B
// row-major per slice, complex64; cmask = C positions of the m bits.
struct NarrowDesc {
  const float2* A;
  const float2* B;
  float2* C;
  int64_t sA, sB, sC;
  int32_t m, k, n, nb;
  uint64_t cmask;
  uint32_t* scale_c;  // per-slice max slots of C, or null
  int32_t cfg;        // 0: LDS-staged tiles; 1: one thread per row (k, n <= 4, m >= 8)
  // filled by launch_narrow
  int32_t q, a_elems;
  uint64_t tmask, rt, nt;
};
bool narrow_fits(int m, int k, int n);
bool narrow_rows_fits(int m, int k, int n);
void launch_narrow(const NarrowDesc& d, hipStream_t st);

// Steps with few outputs and a long sum (m, n <= 3): C[merge(m, n)] =
// sum_k A[m 2^k + k] B[n 2^k + k] with the sum split into chunks of
// 2^kc_bits; FP32 partial sums per chunk, then an FP64 sum over the chunks.
struct SkinnyDesc {
  const float2* A;
  const float2* B;
  float2* C;
  int64_t sA, sB, sC;
  int32_t m, k, n;
  uint64_t cmask;      // output bit j from A's next free bit if (cmask >> j) & 1
  int32_t nb;
  float2* part;        // scratch: [nb][chunks][2^(m+n)] partial sums
  uint32_t* scale_c;   // if set: record the output's per-slice max |x|
};
bool skinny_fits(int m, int k, int n);
int skinny_chunk_bits(int k);  // log2 of the chunk length
// scratch elements (complex64) per slice for a step
int64_t skinny_part_elems(int m, int k, int n);
void launch_skinny(const SkinnyDesc& d, hipStream_t st);

// Fused sub-path (secondary slicing): piece (b, sigma) reads the contiguous
// 2^a elements of T_0 at sigma << a, runs the stages in LDS and writes W_L
// to T_L at pdep(sigma, sig_out) | pdep(w, w_out).
constexpr int kFusedMaxStages = 16;
struct FusedStage {
  const float2* Y;  // small operand, slice 0
  int64_t sY;       // slice stride (elements)
  int32_t m, k, n, yoff;  // yoff: element offset of Y in the LDS copy
  uint64_t cmask;   // positions in W_j of the bits from W_{j-1}
};
struct FusedDesc {
  const float2* X0;
  float2* XL;
  int64_t sX0, sXL;
  int32_t a, nsig, c, rmax, y_elems, nstages, nb, pad;
  uint64_t sig_out, w_out;
  uint32_t* scale_c;  // per-slice max slots of T_L, or null
  FusedStage st[kFusedMaxStages];
};
void launch_fused(const FusedDesc& d, hipStream_t st);

int gemm_config_count(int mode);
bool gemm_config_fits(int cfg, int m, int k, int n, int mode);
const char* gemm_config_name(int cfg, int mode);
void launch_cgemm(const GemmDesc& d, int mode, hipStream_t st);
// Split-K complex64 MFMA GEMM for steps with a long sum and few outputs
// per slice (tiles down to 16 complex columns): blocks take a tile and one
// chunk of the sum and write FP32 partials; a second pass adds the chunks
// in a fixed order and writes C (and its per-slice max when scale_c is set).
int splitk_config_count();
bool splitk_config_fits(int cfg, int m, int k, int n);
const char* splitk_config_name(int cfg);
int splitk_chunk_bits(int m, int k, int n);  // log2 of the number of chunks (0: not offered)
int64_t splitk_part_elems(int m, int k, int n);  // partial elements per slice
void launch_cgemm_splitk(const GemmDesc& d, hipStream_t st);
// complex64 tensor X (2^rank per slice, rank >= 2) -> its split-layout
// copy Y in the given split mode (fp16 scaled by the per-slice max slot[b]).
void launch_split_convert(const float2* X, float2* Y, int rank, int nb, const uint32_t* slot,
                          int mode, hipStream_t st);

}  // namespace ltn
