// Block-sparse (BSR, 32x32 FP32 blocks) purification step and driver for gfx950.
//
// Per product, for operands A, B (symmetric patterns, every diagonal block present; A = B = X
// for a square, A = S2 = Xs^2 and B = X for the second product of Algorithm 1):
//   1. bsr_bitmap_kernel    per block row: bitmap of its block columns + prefix popcounts,
//                           so block (K, c) is found at row_ptr[K] + rank_K(c) in O(1).
//   2. bsr_symbolic_kernel  candidate pattern of A.B: row I = OR of the bitmaps of B's rows
//                           K over the blocks (I, K) of A (integer work).
//   3. bsr_tile_flags       128x128 super-tiles (4x4 blocks) of the upper triangle that hold
//                           a candidate block.
//   4. bsr_product_kernel   one workgroup per super-tile: an f32-MFMA 128x128 tile engine
//                           whose k-stages are the block columns K present in both row
//                           unions; stage K gathers blocks (I_a, K) of A's block rows I_a and
//                           (J_b, K) of B's block rows J_b (B symmetric: B_{K,J} = B_{J,K}^T),
//                           so every operand comes from the super-tile's own 8 block rows,
//                           read in column order, and sits in LDS with its k values
//                           contiguous; zero when absent.  With norm screening
//                           (bsr_block_norms_kernel first, for each operand), a block pair
//                           whose norm product is below the threshold is left out as if
//                           absent.  Fused epilogue:
//                           Y = c2 P + c1 L + c0 I (L = X, or S2), FP64 sums, block norms;
//                           upper blocks written with their transposed mirror.
//   5. bsr_truncate_kernel  keep (I,J) and (J,I) iff ||Y_IJ||_F >= tau (diagonal always; tau
//                           = 0 for Algorithm 1's intermediate S2); ranks in row order;
//                           per-row FP64 sum of kept squared norms.
//   6. bsr_compact_kernel   copy the kept blocks into the next X.
//   7. the dense path's schedule kernel (same on-device scalar state machine).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "schedule_math.h"
#include "snf_internal.h"

namespace snf {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kB = 32;            // block size
constexpr int kBB = kB * kB;      // values per block
constexpr int kSup = 4;           // blocks per super-tile side (128 = 4 x 32)

__device__ __forceinline__ double bsr_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// position of block (row, c) or -1, from the row's bitmap and prefix popcounts
__device__ __forceinline__ int bsr_find(const int32_t* __restrict__ row_ptr,
                                        const uint32_t* __restrict__ bm,
                                        const int32_t* __restrict__ pre, int W, int row, int c) {
  const uint32_t word = bm[(size_t)row * W + (c >> 5)];
  const uint32_t bit = 1u << (c & 31);
  if (!(word & bit)) return -1;
  return row_ptr[row] + pre[(size_t)row * W + (c >> 5)] + __popc(word & (bit - 1u));
}

// ---- 1. bitmaps -------------------------------------------------------------------------
__global__ __launch_bounds__(64) void bsr_bitmap_kernel(const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col_idx,
                                                        int W, uint32_t* __restrict__ bm,
                                                        int32_t* __restrict__ pre) {
  extern __shared__ uint32_t words[];
  const int I = blockIdx.x;
  for (int w = threadIdx.x; w < W; w += blockDim.x) words[w] = 0u;
  __syncthreads();
  for (int p = row_ptr[I] + threadIdx.x; p < row_ptr[I + 1]; p += blockDim.x) {
    const int c = col_idx[p];
    atomicOr(&words[c >> 5], 1u << (c & 31));
  }
  __syncthreads();
  for (int w = threadIdx.x; w < W; w += blockDim.x) bm[(size_t)I * W + w] = words[w];
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < W; ++w) {
      pre[(size_t)I * W + w] = s;
      s += __popc(words[w]);
    }
  }
}

// ---- 2. symbolic ------------------------------------------------------------------------
// Pattern of A.B (both symmetric patterns): row I is the OR of the bitmaps of B's block rows
// K over the blocks (I, K) of A.
__global__ __launch_bounds__(64) void bsr_symbolic_kernel(const int32_t* __restrict__ row_ptrA,
                                                          const int32_t* __restrict__ colA,
                                                          const int32_t* __restrict__ row_ptrB,
                                                          const uint32_t* __restrict__ bm, int W,
                                                          const int32_t* __restrict__ pre,
                                                          uint32_t* __restrict__ bmP,
                                                          int32_t* __restrict__ preP,
                                                          int32_t* __restrict__ cntP,
                                                          int64_t* __restrict__ triples) {
  extern __shared__ uint32_t acc[];
  const int I = blockIdx.x;
  for (int w = threadIdx.x; w < W; w += blockDim.x) acc[w] = 0u;
  int64_t tri = 0;   // block triples (I, K, J), J >= I: the useful work of row I
  for (int p = row_ptrA[I]; p < row_ptrA[I + 1]; ++p) {
    const int K = colA[p];
    for (int w = threadIdx.x; w < W; w += blockDim.x) acc[w] |= bm[(size_t)K * W + w];
    if (threadIdx.x == 0) {
      const uint32_t word = bm[(size_t)K * W + (I >> 5)];
      const int below = pre[(size_t)K * W + (I >> 5)] + __popc(word & ((1u << (I & 31)) - 1u));
      tri += (row_ptrB[K + 1] - row_ptrB[K]) - below;
    }
  }
  if (threadIdx.x == 0) triples[I] = tri;
  __syncthreads();
  for (int w = threadIdx.x; w < W; w += blockDim.x) bmP[(size_t)I * W + w] = acc[w];
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < W; ++w) {
      preP[(size_t)I * W + w] = s;
      s += __popc(acc[w]);
    }
    cntP[I] = s;
  }
}

__global__ __launch_bounds__(64) void bsr_fill_cols_kernel(const uint32_t* __restrict__ bmP,
                                                           const int32_t* __restrict__ preP,
                                                           const int32_t* __restrict__ row_ptrP,
                                                           int W, int32_t* __restrict__ colP) {
  const int I = blockIdx.x;
  for (int w = threadIdx.x; w < W; w += blockDim.x) {
    uint32_t bits = bmP[(size_t)I * W + w];
    int pos = row_ptrP[I] + preP[(size_t)I * W + w];
    while (bits) {
      const int b = __ffs(bits) - 1;
      colP[pos++] = w * 32 + b;
      bits &= bits - 1u;
    }
  }
}

// ---- 3. super-tiles ---------------------------------------------------------------------
__global__ void bsr_tile_flags_kernel(const uint32_t* __restrict__ bmP, int nb, int W, int NT,
                                      uint8_t* __restrict__ flags) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)NT * NT) return;
  const int TI = (int)(t / NT), TJ = (int)(t % NT);
  uint8_t f = 0;
  if (TI <= TJ) {
    const int c0 = kSup * TJ;
    const uint32_t mask = 0xFu << (c0 & 31);
    for (int a = 0; a < kSup; ++a) {
      const int I = kSup * TI + a;
      if (I < nb && (bmP[(size_t)I * W + (c0 >> 5)] & mask)) f = 1;
    }
  }
  flags[t] = f;
}

// ---- 4. numeric product -----------------------------------------------------------------
struct BsrMat {                    // device view of one BSR matrix with its lookup tables
  const int32_t* row_ptr;
  const uint32_t* bm;
  const int32_t* pre;
  float* val;
};

struct BsrProductArgs {
  BsrMat X;            // left operand A (A_IK is read from block row I)
  BsrMat Y;            // right operand B (the same matrix as X for a square); symmetric:
                       // B_KJ is read as the transpose of B_JK, from block row J
  BsrMat L;            // linear term of the epilogue (X for a square; S2 for Algorithm 1's
                       // second product)
  BsrMat P;            // candidate pattern of the output, values written here
  float* val2;         // second output d2 P + d1 L + d0 I over the same candidate pattern
                       // (the first product of a P_{i,j} iteration), or null
  double* normP;       // squared Frobenius norm per candidate block
  const int32_t* tiles;  // (TI << 16) | TJ
  double* partials;    // [tiles][4]
  const double* nrmX;  // squared Frobenius norm per block of A (screening only)
  const double* nrmY;  // the same for B (nrmX when B is A)
  double screen2;      // screening threshold squared; 0: no screening
  int nb, W;
};

// Squared Frobenius norm of every block of X in FP64, one wave per block (lane l sums the
// squares of its 16 values in order, then a fixed butterfly): the operand norms of the
// product's norm screening.
__global__ __launch_bounds__(256) void bsr_block_norms_kernel(const float* __restrict__ val,
                                                              int64_t nnzb,
                                                              double* __restrict__ nrm2) {
  const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blk >= nnzb) return;                 // uniform across the wave
  const int lane = threadIdx.x & 63;
  const float* p = val + blk * kBB + lane * 4;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < kBB / 256; ++r) {
    const float4 v = *(const float4*)(p + r * 256);
    acc += (double)v.x * v.x;
    acc += (double)v.y * v.y;
    acc += (double)v.z * v.z;
    acc += (double)v.w * v.w;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) nrm2[blk] = acc;
}

constexpr int kBsrLdsK = kB + 4;    // LDS row stride (floats) of a panel row: 32 values of k
                                    // and 4 of padding (16-byte reads of 16 rows hit
                                    // distinct banks)
constexpr int kChunkWords = 8;
// Word 3 of a buffer resource on the gfx9 family (32-bit data format; the value AMD's
// composable_kernel library uses for these parts).  The untyped loads below ignore the
// format; a load at or past the resource's size returns zero.
constexpr int kBufferFlags = 0x00020000;      // bitmap words per k-stage list chunk (256 columns)
static_assert(kChunkWords * 32 <= 256, "a chunk's stages must fit waves 0-3 (compaction)");

// LDS of the numeric kernel, in one struct so that the small per-chunk tables sit at low
// addresses (reachable through the 16-bit offset of the LDS instructions) and the panels
// after them.
struct BsrProductSmem {
  double red[24];
  // per k-stage: the rank of block (row, K) within the chunk's part of each panel row, one
  // byte per row (A rows in krel[0], B rows in krel[1])
  uint32_t krel[2][kChunkWords * 32];
  // the chunk's bitmap words of the 8 panel rows (A rows I_0..I_3, then B rows J_0..J_3) and
  // the value index of the first block of each word (row_ptr + prefix count)
  uint32_t bmc[2 * kSup][kChunkWords];
  int32_t prc[2 * kSup][kChunkWords];
  int offs[1];                  // stages of the chunk
  int wkeep[4];                 // stages kept per wave (screening)
  uint32_t spres[2];
  uint16_t klist[kChunkWords * 32];
  // per k-stage: the block pairs (A block a, B block b) the stage multiplies, bit 4 a + b
  // (both present and, with screening, norm product at or above the threshold)
  uint16_t kmask[kChunkWords * 32];
  // panels of stage K: row 32 a + i holds row i of block (I_a, K) (A side) or (J_b, K)
  // (B side), its 32 values of k contiguous
  __attribute__((aligned(16))) float sA[2][kSup * kB][kBsrLdsK];
  __attribute__((aligned(16))) float sB[2][kSup * kB][kBsrLdsK];
};

// 512 threads, at least 4 waves per SIMD (two workgroups per compute unit: <= 128 VGPRs)
__global__ __launch_bounds__(512, 4) void bsr_product_kernel(const SnfState* __restrict__ st,
                                                             BsrProductArgs g) {
  if (st->stop) return;
  __shared__ BsrProductSmem sm;

  const int packed = g.tiles[blockIdx.x];
  const int TI = packed >> 16, TJ = packed & 0xFFFF;
  const int W = g.W, nb = g.nb;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // waves w and w + 4 share a SIMD (waves go to the SIMDs in turn): give them opposite A
  // rows (0/3, 1/2) and opposite B pairs, so a stage whose blocks are present on one side of
  // the super-tile only still spreads its MFMAs over all four SIMDs
  const int wr = wid < 4 ? (wid >> 1) : 3 - ((wid - 4) >> 1);
  const int wc = wid < 4 ? (wid & 1) : 1 - ((wid - 4) & 1);
  const int ci0 = kSup * TI, cj0 = kSup * TJ;   // first block row of the A / B panels

  // 8 waves: wave (wr, wc) holds A block row wr (32 rows) against B blocks 2 wc, 2 wc + 1
  flt4 acc[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[m][q] = flt4{0.f, 0.f, 0.f, 0.f};

  // Wave wid moves one block of the stage: side wid / 4 (A, B), block ab = wid % 4, i.e. block
  // (I_ab, K) of A's row I_ab or (J_ab, K) of B's row J_ab (A_{I,K} is that block itself; B is
  // symmetric, so B_{K,J} is the transpose of block (J, K)).  Lane l moves the 16-byte pieces
  // l + 64 q (q = 0..3): row (l / 8) + 8 q, values of k 4 (l % 8) .. + 3.
  const int side = wid >> 2, ab = wid & 3, prow = side * kSup + ab;
  const float* valS = side ? g.Y.val : g.X.val;   // this wave's operand
  const int lrow = lane >> 3, lcol = 4 * (lane & 7);
  u32x4 rA[4], rB[4];
  uint32_t pA = 0, pB = 0;   // block pairs of the stage (kmask)
  int rowbase = 0;           // value index of the first block of this wave's row in the chunk
  auto gload = [&](int s, int nk, u32x4 (&rv)[4], uint32_t& pres) {
    // The block is loaded when some pair of the stage uses it.  The four loads are buffer
    // loads issued on every path: for a block no pair uses, or a stage past the end, the
    // buffer's size is 0 and they return zeros without touching memory.  So the number of
    // loads in flight is the same on every path, and the wait before a stage's LDS stores
    // leaves the next stage's loads in flight.  (The stage tables are the same for every
    // lane: read as wave-uniform values.)
    const int si = min(s, nk - 1);
    const uint32_t m = s < nk ? __builtin_amdgcn_readfirstlane(sm.kmask[si]) : 0u;
    pres = m;
    const uint32_t need = side ? ((m | (m >> 4) | (m >> 8) | (m >> 12)) >> ab) & 1u
                               : (((m >> (4 * ab)) & 0xFu) != 0u ? 1u : 0u);
    const int pos =
        rowbase + (int)((__builtin_amdgcn_readfirstlane(sm.krel[side][si]) >> (8 * ab)) & 0xFFu);
    const uint64_t addr = (uint64_t)(need ? valS + (size_t)pos * kBB : valS);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)addr);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
    const int bytes = __builtin_amdgcn_readfirstlane(need ? kBB * 4 : 0);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(((uint64_t)hi << 32) | lo), 0, bytes, kBufferFlags);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      rv[q] = __builtin_bit_cast(
          u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * lane + 1024 * q, 0, 0));
  };
  auto lstore = [&](int buf, const u32x4 (&rv)[4], uint32_t pres) {
    float(*dst)[kBsrLdsK] = side ? sm.sB[buf] : sm.sA[buf];
#pragma unroll
    for (int q = 0; q < 4; ++q) *(u32x4*)(&dst[ab * kB + lrow + 8 * q][lcol]) = rv[q];
    if (tid == 0) sm.spres[buf] = pres;
  };

  // MFMA operands: lane (fr, fk) takes row fr of its 16-row piece at k = 8 fk + t in step t
  // (t = 0..7; each step sums over the four fk), read as two 16-byte pieces.  The products
  // of B blocks q0 / 2 .. (q1 - 1) / 2 of this wave's pair.
  const int fr = lane & 15, fk = lane >> 4;
  auto mfma_pairs = [&](int buf, auto q0c, auto q1c) {
    constexpr int q0 = decltype(q0c)::value, q1 = decltype(q1c)::value;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      flt4 a[2], b[4];
#pragma unroll
      for (int m = 0; m < 2; ++m)
        a[m] = *(const flt4*)(&sm.sA[buf][wr * kB + m * 16 + fr][8 * fk + 4 * h]);
#pragma unroll
      for (int q = q0; q < q1; ++q)
        b[q] = *(const flt4*)(&sm.sB[buf][wc * 64 + q * 16 + fr][8 * fk + 4 * h]);
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int q = q0; q < q1; ++q)
#pragma unroll
          for (int m = 0; m < 2; ++m)
            acc[m][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m][tt], b[q][tt], acc[m][q], 0, 0, 0);
      // the second half's reads stay behind the first half's MFMAs (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  auto compute = [&](int buf) {
    // this wave's A block (row wr) and two B blocks; the MFMAs of pairs the stage leaves
    // out (a block absent, or screened) are skipped (uniform across the wave)
    const uint32_t pm = __builtin_amdgcn_readfirstlane(sm.spres[buf]);
    const uint32_t pp = (pm >> (4 * wr + 2 * wc)) & 3u;
    if (pp == 3u)
      mfma_pairs(buf, std::integral_constant<int, 0>(), std::integral_constant<int, 4>());
    else if (pp == 1u)
      mfma_pairs(buf, std::integral_constant<int, 0>(), std::integral_constant<int, 2>());
    else if (pp == 2u)
      mfma_pairs(buf, std::integral_constant<int, 2>(), std::integral_constant<int, 4>());
  };
  // k-stages: block columns K present in both (rows I_a) and (rows J_b), taken in chunks
  // of kChunkWords bitmap words
  // Wave 0 holds the bitmap word and the value index base of (panel row lane / 8, word
  // lane % 8) of the next chunk; it fetches them while the current chunk's stages run.
  uint32_t nword = 0u;
  int nbase = 0;
  auto fetch_rows = [&](int w0n) {
    const int r = lane >> 3, w = w0n + (lane & 7);
    const int row = r < kSup ? ci0 + r : cj0 + (r - kSup);
    nword = 0u;
    nbase = 0;
    if (row < nb && w < W) {
      const BsrMat& M = r < kSup ? g.X : g.Y;
      nword = M.bm[(size_t)row * W + w];
      nbase = M.row_ptr[row] + M.pre[(size_t)row * W + w];
    }
  };
  if (wid == 0) fetch_rows(0);
  for (int w0 = 0; w0 < W; w0 += kChunkWords) {
    __syncthreads();                       // the previous chunk is done with its tables / LDS
    if (wid == 0) {
      // the chunk's words, the stage list (the columns set in the union of the A rows and in
      // the union of the B rows, ascending), then the next chunk's words
      sm.bmc[lane >> 3][lane & 7] = nword;
      sm.prc[lane >> 3][lane & 7] = nbase;
      uint32_t u = nword;
      u |= __shfl_xor(u, 8);
      u |= __shfl_xor(u, 16);              // OR over the 4 rows of this lane's side
      const uint32_t sw = u & __shfl_xor(u, 32);
      const int cnt = __popc(sw);
      int incl = cnt;                      // inclusive prefix over the 8 words (lanes 0-7)
#pragma unroll
      for (int o = 1; o < kChunkWords; o <<= 1) {
        const int v = __shfl_up(incl, o, kChunkWords);
        if ((lane & (kChunkWords - 1)) >= o) incl += v;
      }
      if (lane < kChunkWords) {
        uint32_t bits = sw;
        int pos = incl - cnt;
        while (bits) {
          const int b = __ffs(bits) - 1;
          sm.klist[pos++] = (uint16_t)((w0 + lane) * 32 + b);
          bits &= bits - 1u;
        }
        if (lane == kChunkWords - 1) sm.offs[0] = incl;
      }
      if (w0 + kChunkWords < W) fetch_rows(w0 + kChunkWords);
    }
    __syncthreads();
    int nk = sm.offs[0];
    rowbase = __builtin_amdgcn_readfirstlane(sm.prc[prow][0]);
    for (int t = tid; t < nk; t += 512) {
      const int K = sm.klist[t];
      const int wl = (K >> 5) - w0;
      const uint32_t lo = (1u << (K & 31)) - 1u, bit = 1u << (K & 31);
      uint32_t ba = 0u, bb = 0u, ra = 0u, rb = 0u;
      int pa[kSup], pb[kSup];
#pragma unroll
      for (int a = 0; a < kSup; ++a) {
        const uint32_t wa = sm.bmc[a][wl], wb = sm.bmc[kSup + a][wl];
        // rank within the chunk: below 32 * kChunkWords = 256, one byte
        const int qa = sm.prc[a][wl] - sm.prc[a][0] + __popc(wa & lo);
        const int qb = sm.prc[kSup + a][wl] - sm.prc[kSup + a][0] + __popc(wb & lo);
        ba |= (wa & bit) ? (1u << a) : 0u;
        bb |= (wb & bit) ? (1u << a) : 0u;
        ra |= (uint32_t)(qa & 0xFF) << (8 * a);
        rb |= (uint32_t)(qb & 0xFF) << (8 * a);
        pa[a] = sm.prc[a][0] + qa;
        pb[a] = sm.prc[kSup + a][0] + qb;
      }
      uint32_t m = 0u;
#pragma unroll
      for (int a = 0; a < kSup; ++a)
        if ((ba >> a) & 1u) m |= bb << (4 * a);
      if (g.screen2 > 0.0 && m) {
        double na[kSup], nbv[kSup];
#pragma unroll
        for (int a = 0; a < kSup; ++a) {
          na[a] = ((ba >> a) & 1u) ? g.nrmX[pa[a]] : 0.0;
          nbv[a] = ((bb >> a) & 1u) ? g.nrmY[pb[a]] : 0.0;
        }
        uint32_t drop = 0u;
#pragma unroll
        for (int a = 0; a < kSup; ++a) {
          uint32_t da = 0u;
#pragma unroll
          for (int b = 0; b < kSup; ++b) da |= na[a] * nbv[b] < g.screen2 ? (1u << b) : 0u;
          drop |= da << (4 * a);
        }
        m &= ~drop;
      }
      sm.krel[0][t] = ra;
      sm.krel[1][t] = rb;
      sm.kmask[t] = (uint16_t)m;
    }
    __syncthreads();
    if (g.screen2 > 0.0) {
      // drop the stages whose every pair is screened out, keeping the order of the rest
      // (nk <= kChunkWords * 32 = 256: thread t < nk holds stage t)
      const bool keep = tid < nk && sm.kmask[tid] != 0;
      const unsigned long long bal = __ballot(keep);
      if (lane == 0 && wid < 4) sm.wkeep[wid] = __popcll(bal);
      uint32_t era = 0u, erb = 0u;
      uint16_t em = 0;
      if (keep) {
        era = sm.krel[0][tid];
        erb = sm.krel[1][tid];
        em = sm.kmask[tid];
      }
      __syncthreads();                     // every entry read before any is overwritten
      if (keep) {
        int pos = __popcll(bal & ((1ull << lane) - 1ull));
        for (int v = 0; v < wid; ++v) pos += sm.wkeep[v];
        sm.krel[0][pos] = era;
        sm.krel[1][pos] = erb;
        sm.kmask[pos] = em;
      }
      nk = sm.wkeep[0] + sm.wkeep[1] + sm.wkeep[2] + sm.wkeep[3];
      __syncthreads();
    }
    if (nk == 0) continue;
    // two stages in flight in registers: stage s in LDS buffer s & 1, s + 1 loaded into
    // registers, s + 2 being loaded
    gload(0, nk, rA, pA);
    gload(1, nk, rB, pB);
    lstore(0, rA, pA);
    __syncthreads();
    for (int s = 0; s < nk; s += 2) {
      gload(s + 2, nk, rA, pA);
      compute(0);
      if (s + 1 < nk) lstore(1, rB, pB);
      __syncthreads();
      if (s + 1 >= nk) break;
      gload(s + 3, nk, rB, pB);
      compute(1);
      if (s + 2 < nk) lstore(0, rA, pA);
      __syncthreads();
    }
  }

  // Epilogue.  Wave (wr, wc) holds blocks (wr, 2 wc + bj) of the super-tile; the f32 MFMA
  // accumulator of lane l, register v is row 4 (l / 16) + v, column l % 16 of its 16x16
  // piece (m, q): rows m 16 + ... of block row wr, block bj = q / 2.
  const double c2 = st->c2, c1 = st->c1, c0 = st->c0;
  const double d2 = st->d2, d1 = st->d1, d0 = st->d0;
  const int want_e = st->want_e;
  double e2 = 0.0, t1 = 0.0;
  {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int I = kSup * TI + wr, J = kSup * TJ + 2 * wc + bj;
      if (I >= nb || J >= nb) continue;
      if (I > J) continue;                       // lower blocks come from their mirror
      const int pp = bsr_find(g.P.row_ptr, g.P.bm, g.P.pre, W, I, J);
      if (pp < 0) continue;                      // no candidate: nothing contributes
      const int ppT = (I == J) ? pp : bsr_find(g.P.row_ptr, g.P.bm, g.P.pre, W, J, I);
      const int px = bsr_find(g.L.row_ptr, g.L.bm, g.L.pre, W, I, J);
      float* Y = g.P.val + (size_t)pp * kBB;
      float* YT = g.P.val + (size_t)ppT * kBB;
      float* Y2 = g.val2 ? g.val2 + (size_t)pp * kBB : nullptr;
      float* YT2 = g.val2 ? g.val2 + (size_t)ppT * kBB : nullptr;
      const float* Xb = px >= 0 ? g.L.val + (size_t)px * kBB : nullptr;
      double nrm2 = 0.0;
#pragma unroll
      for (int mm = 0; mm < 2; ++mm) {
#pragma unroll
        for (int qq = 0; qq < 2; ++qq) {
          const int m = mm, q = 2 * bj + qq;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = mm * 16 + 4 * (lane >> 4) + v;
            const int c = qq * 16 + (lane & 15);
            if (I == J && r > c) continue;       // diagonal block: upper half, mirrored
            const bool mirror = (I != J) || (r != c);
            const double w = mirror ? 2.0 : 1.0;
            const double p = (double)acc[m][q][v];
            const double x = Xb ? (double)Xb[r * kB + c] : 0.0;
            if (want_e) {
              const double d = p - x;
              e2 += w * (d * d);
            }
            const double y = c2 * p + c1 * x + ((I == J && r == c) ? c0 : 0.0);
            if (I == J && r == c) t1 += y;
            const float yf = (float)y;
            nrm2 += (I == J ? w : 1.0) * ((double)yf * (double)yf);
            Y[r * kB + c] = yf;
            if (mirror) YT[c * kB + r] = yf;
            if (Y2) {
              const float y2 = (float)(d2 * p + d1 * x + ((I == J && r == c) ? d0 : 0.0));
              Y2[r * kB + c] = y2;
              if (mirror) YT2[c * kB + r] = y2;
            }
          }
        }
      }
      nrm2 = bsr_wave_sum(nrm2);
      if (lane == 0) {
        g.normP[pp] = nrm2;
        g.normP[ppT] = nrm2;
      }
    }
  }
  // block_sum of e2, t1 (fixed order)
  double t2 = 0.0;
  e2 = bsr_wave_sum(e2);
  t1 = bsr_wave_sum(t1);
  if (lane == 0) {
    sm.red[wid * 3 + 0] = e2;
    sm.red[wid * 3 + 1] = t1;
    sm.red[wid * 3 + 2] = t2;
  }
  __syncthreads();
  if (tid == 0) {
    double se = 0.0, st1 = 0.0;
    for (int k = 0; k < 8; ++k) {       // wave order
      se += sm.red[k * 3 + 0];
      st1 += sm.red[k * 3 + 1];
    }
    g.partials[blockIdx.x * 4 + 0] = se;
    g.partials[blockIdx.x * 4 + 1] = st1;
    g.partials[blockIdx.x * 4 + 2] = 0.0;
    g.partials[blockIdx.x * 4 + 3] = 0.0;
  }
}

// ---- 5. truncation ----------------------------------------------------------------------
// One workgroup per block row; thread 0 walks the row in order (ranks and the FP64 sum of
// kept squared norms in a fixed order).
__global__ __launch_bounds__(64) void bsr_truncate_kernel(const int32_t* __restrict__ row_ptrP,
                                                          const int32_t* __restrict__ colP,
                                                          const double* __restrict__ normP,
                                                          double tau2, int32_t* __restrict__ rank,
                                                          int32_t* __restrict__ cnt,
                                                          double* __restrict__ partials,
                                                          int slot0) {
  const int I = blockIdx.x;
  if (threadIdx.x != 0) return;
  int k = 0;
  double t2 = 0.0;
  for (int p = row_ptrP[I]; p < row_ptrP[I + 1]; ++p) {
    const bool keep = (colP[p] == I) || (normP[p] >= tau2);
    rank[p] = keep ? k : -1;
    if (keep) {
      ++k;
      t2 += normP[p];
    }
  }
  cnt[I] = k;
  partials[(slot0 + I) * 4 + 0] = 0.0;
  partials[(slot0 + I) * 4 + 1] = 0.0;
  partials[(slot0 + I) * 4 + 2] = t2;
  partials[(slot0 + I) * 4 + 3] = 0.0;
}

// ---- 5a. error-controlled truncation: histogram of block norms ------------------------
// Half-octave bins of the squared block norm s: bin(s) = floor(2 log2 s), exact from the
// binary exponent and the mantissa against fl(sqrt 2) (no double lies between sqrt 2 and
// fl(sqrt 2), so the comparison is exact), clamped to [kBinMin, kBinMax]; s = 0 -> kBinMin.
constexpr int kBinMin = -160, kBinMax = 40, kNumBins = kBinMax - kBinMin + 1;
constexpr double kSqrt2 = 1.4142135623730951;

__device__ __forceinline__ int half_octave_bin(double s) {
  if (!(s > 0.0)) return kBinMin;
  int e = 0;
  const double m = frexp(s, &e);                 // s = m 2^e, m in [0.5, 1)
  const int j = 2 * (e - 1) + (2.0 * m >= kSqrt2 ? 1 : 0);
  return j < kBinMin ? kBinMin : (j > kBinMax ? kBinMax : j);
}

// Counts of the candidate blocks (I, J), J > I, per bin (each stands for a mirror pair).
// Integer atomics: the counts do not depend on the order of arrival.
__global__ __launch_bounds__(64) void bsr_norm_hist_kernel(const int32_t* __restrict__ row_ptrP,
                                                           const int32_t* __restrict__ colP,
                                                           const double* __restrict__ normP,
                                                           uint32_t* __restrict__ counts) {
  __shared__ uint32_t h[kNumBins];
  for (int b = threadIdx.x; b < kNumBins; b += 64) h[b] = 0u;
  __syncthreads();
  const int I = blockIdx.x;
  for (int p = row_ptrP[I] + (int)threadIdx.x; p < row_ptrP[I + 1]; p += 64)
    if (colP[p] > I) atomicAdd(&h[half_octave_bin(normP[p]) - kBinMin], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < kNumBins; b += 64)
    if (h[b]) atomicAdd(&counts[b], h[b]);
}

// Squared-norm threshold of the error-controlled rule from the bin counts: the lowest bins
// are dropped while their charge, 2 count_j 2^((j+1)/2) summed (each bin at its upper edge,
// mirror blocks included), stays within eps_i^2.  Returns tau2 such that a block is kept iff
// its squared norm >= tau2 (0: keep all; +inf: drop every off-diagonal block).
static double error_control_tau2(const uint32_t* counts, double eps_i) {
  const double budget = eps_i * eps_i;
  double charge = 0.0;
  int k = kBinMin;
  for (int j = kBinMin; j <= kBinMax; ++j) {
    const double wj = 2.0 * (double)counts[j - kBinMin];
    if (wj == 0.0) {
      k = j + 1;
      continue;
    }
    const double c = wj * pow(2.0, (j + 1) / 2.0);
    if (charge + c > budget) {
      k = j;
      break;
    }
    charge += c;
    k = j + 1;
  }
  if (k <= kBinMin) return 0.0;
  if (k > kBinMax) return INFINITY;
  // bin(s) >= k  <=>  s >= 2^(k/2) (k even), s >= fl(sqrt 2) 2^((k-1)/2) (k odd)
  return (k % 2 == 0) ? ldexp(1.0, k / 2) : ldexp(kSqrt2, (k - 1) / 2);
}

// ---- 6. compaction ----------------------------------------------------------------------
__global__ __launch_bounds__(256) void bsr_compact_kernel(const int32_t* __restrict__ row_ptrP,
                                                          const int32_t* __restrict__ colP,
                                                          const float* __restrict__ valP,
                                                          const int32_t* __restrict__ rank,
                                                          const int32_t* __restrict__ row_ptrN,
                                                          int32_t* __restrict__ colN,
                                                          float* __restrict__ valN) {
  const int I = blockIdx.x;
  for (int p = row_ptrP[I]; p < row_ptrP[I + 1]; ++p) {
    const int k = rank[p];
    if (k < 0) continue;
    const int dst = row_ptrN[I] + k;
    if (threadIdx.x == 0) colN[dst] = colP[p];
    const u32x4 v = *(const u32x4*)(valP + (size_t)p * kBB + threadIdx.x * 4);
    *(u32x4*)(valN + (size_t)dst * kBB + threadIdx.x * 4) = v;
  }
}

// ---- f0 on blocks -----------------------------------------------------------------------
// Copy of X that reads only its upper blocks (I <= J, upper half of diagonal blocks): every
// lower block is written as the transpose of its mirror, so the copy is exactly symmetric
// (the numeric kernel reads both halves of the block rows of its super-tile).
__global__ __launch_bounds__(256) void bsr_sym_copy_kernel(const int32_t* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ col,
                                                           const uint32_t* __restrict__ bm,
                                                           const int32_t* __restrict__ pre,
                                                           int W, const float* __restrict__ vin,
                                                           float* __restrict__ vout, int nbrows) {
  for (int I = blockIdx.x; I < nbrows; I += gridDim.x) {
    for (int p = row_ptr[I]; p < row_ptr[I + 1]; ++p) {
      const int J = col[p];
      const int src = (I <= J) ? p : bsr_find(row_ptr, bm, pre, W, J, I);
      for (int e = threadIdx.x; e < kBB; e += blockDim.x) {
        const int r = e / kB, c = e % kB;
        const bool direct = I < J || (I == J && r <= c);
        vout[(size_t)p * kBB + e] = direct ? vin[(size_t)src * kBB + r * kB + c]
                                           : vin[(size_t)src * kBB + c * kB + r];
      }
    }
  }
}

// X_0 = (lambda_max I - F)/(lambda_max - lambda_min), block by block, reading only F's
// upper blocks (I <= J, upper half of diagonal blocks) and mirroring.
__global__ __launch_bounds__(256) void bsr_f0_kernel(const int32_t* __restrict__ row_ptrF,
                                                     const int32_t* __restrict__ colF,
                                                     const uint32_t* __restrict__ bmF,
                                                     const int32_t* __restrict__ preF,
                                                     const float* __restrict__ valF, int W,
                                                     const SnfState* __restrict__ st,
                                                     float* __restrict__ valX,
                                                     double* __restrict__ partials, int nbrows) {
  __shared__ double red[12];
  const double lmin = st->lambda_min, lmax = st->lambda_max;
  // fixed-mu schemes (Algorithm 1, McWeeny, P_{m,m}, P_{i,j}): X_0 = (mu I - F) / gamma +
  // x* I (x* = 1/2 but for P_{i,j}); else Algorithm 2's map
  const bool alg1 = st->scheme == SNF_SNF_FIXMU || st->scheme == SNF_MCWEENY || st->pmm_m ||
                    st->pij_i;
  const double mu = st->mu, gamma = st->gamma, xs = st->xstar;
  double t1 = 0.0, t2 = 0.0;
  // grid-stride over block rows; every thread handles 4 values of each block
  for (int I = blockIdx.x; I < nbrows; I += gridDim.x) {
    for (int p = row_ptrF[I]; p < row_ptrF[I + 1]; ++p) {
      const int J = colF[p];
      const int src = (I <= J) ? p : bsr_find(row_ptrF, bmF, preF, W, J, I);
      for (int e = threadIdx.x; e < kBB; e += blockDim.x) {
        const int r = e / kB, c = e % kB;
        float fv;
        if (I < J) fv = valF[(size_t)src * kBB + r * kB + c];
        else if (I > J) fv = valF[(size_t)src * kBB + c * kB + r];
        else fv = (r <= c) ? valF[(size_t)src * kBB + r * kB + c] : valF[(size_t)src * kBB + c * kB + r];
        const bool d = (I == J && r == c);
        const double x = alg1 ? ((d ? mu : 0.0) - (double)fv) / gamma + (d ? xs : 0.0)
                              : ((d ? lmax : 0.0) - (double)fv) / (lmax - lmin);
        const float xf = (float)x;
        valX[(size_t)p * kBB + e] = xf;
        if (d) t1 += (double)xf;
        t2 += (double)xf * (double)xf;
      }
    }
  }
  double e0 = 0.0;
  // fixed-order block sum
  e0 = bsr_wave_sum(e0);
  t1 = bsr_wave_sum(t1);
  t2 = bsr_wave_sum(t2);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid * 3 + 0] = e0;
    red[wid * 3 + 1] = t1;
    red[wid * 3 + 2] = t2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = 0.0;
    partials[blockIdx.x * 4 + 1] = ((red[1] + red[4]) + red[7]) + red[10];
    partials[blockIdx.x * 4 + 2] = ((red[2] + red[5]) + red[8]) + red[11];
    partials[blockIdx.x * 4 + 3] = 0.0;
  }
}

// =========================================================================================
// Host side
// =========================================================================================
static thread_local char g_bsr_err[256];

static int bsr_dev_error(hipError_t e, const char* what) {
  snprintf(g_bsr_err, sizeof(g_bsr_err), "HIP error in %s: %s", what, hipGetErrorString(e));
  return SNF_EDEVICE;
}

#define BSR_HIP(call)                                      \
  do {                                                     \
    hipError_t _e = (call);                                \
    if (_e != hipSuccess) return bsr_dev_error(_e, #call); \
  } while (0)

// Growable device array.
template <typename T>
struct DevArr {
  T* p = nullptr;
  size_t cap = 0;
  int reserve(size_t n) {
    if (n <= cap) return SNF_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    size_t want = n + n / 4 + 16;
    if (hipMalloc(&p, want * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      return SNF_ENOMEM;
    }
    cap = want;
    return SNF_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

struct BsrBuf {                 // one BSR matrix owned by the library, with lookup tables
  DevArr<int32_t> row_ptr, col;
  DevArr<float> val;
  DevArr<uint32_t> bm;
  DevArr<int32_t> pre;
  int64_t nnzb = 0;
  void release() {
    row_ptr.release();
    col.release();
    val.release();
    bm.release();
    pre.release();
    nnzb = 0;
  }
  BsrMat view() const { return BsrMat{row_ptr.p, bm.p, pre.p, val.p}; }
};

struct BsrWorkspace {
  BsrBuf X[2], P, Fl;           // current / next X, candidate product, F's lookup tables
  BsrBuf S, T;                  // the iteration's intermediates (Algorithm 1's S2 = Xs^2;
                                // P_{m,m}'s and P_{i,j}'s W and Horner levels)
  DevArr<float> val2;           // second output of a dual product, candidate pattern
  // the schedule's buffer indices 0..3 (operands, linear term and output of each product)
  BsrBuf& buf(int i) { return i == 0 ? X[0] : i == 1 ? X[1] : i == 2 ? S : T; }
  DevArr<double> normP, partials, sums;
  DevArr<double> nrmX, nrmY;    // norm screening: squared norms of the operands' blocks
  DevArr<int32_t> cnt, rank, tiles;
  DevArr<int64_t> triples;
  int64_t last_triples = 0;
  DevArr<uint8_t> flags;
  SnfState* state = nullptr;
  SnfState* state_host = nullptr;
  int32_t* pinned = nullptr;    // scratch for small read-backs
  size_t pinned_cap = 0;
  DevArr<uint32_t> hist;        // error-controlled truncation: bin counts (device)
  double last_tau2 = 0.0;       // squared-norm threshold the last step used
  uint32_t* hist_host = nullptr;   // pinned copy
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::mutex mu;
};

static std::mutex g_bsr_mu;
static BsrWorkspace* g_bsr_ws[64];

static BsrWorkspace* bsr_workspace() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(g_bsr_mu);
  if (!g_bsr_ws[dev]) g_bsr_ws[dev] = new BsrWorkspace();
  return g_bsr_ws[dev];
}

void bsr_release_all_devices() {
  int prev = 0;
  const bool restore = hipGetDevice(&prev) == hipSuccess;
  for (int dev = 0; dev < 64; ++dev) {
    BsrWorkspace* w = nullptr;
    {
      std::lock_guard<std::mutex> g(g_bsr_mu);
      w = g_bsr_ws[dev];
    }
    if (!w || hipSetDevice(dev) != hipSuccess) continue;
    std::lock_guard<std::mutex> g(w->mu);
    (void)hipDeviceSynchronize();
    for (BsrBuf* b : {&w->X[0], &w->X[1], &w->P, &w->Fl, &w->S, &w->T}) b->release();
    w->normP.release();
    w->partials.release();
    w->sums.release();
    w->nrmX.release();
    w->nrmY.release();
    w->val2.release();
    w->cnt.release();
    w->rank.release();
    w->tiles.release();
    w->triples.release();
    w->flags.release();
    w->hist.release();
    if (w->state) (void)hipFree(w->state);
    w->state = nullptr;
    if (w->state_host) (void)hipHostFree(w->state_host);
    w->state_host = nullptr;
    if (w->pinned) (void)hipHostFree(w->pinned);
    w->pinned = nullptr;
    w->pinned_cap = 0;
    if (w->hist_host) (void)hipHostFree(w->hist_host);
    w->hist_host = nullptr;
    for (int i = 0; i < 4; ++i) {
      if (w->ev[i]) (void)hipEventDestroy(w->ev[i]);
      w->ev[i] = nullptr;
    }
  }
  if (restore) (void)hipSetDevice(prev);
}

static int ensure_pinned(BsrWorkspace* w, size_t bytes) {
  if (bytes <= w->pinned_cap) return SNF_OK;
  if (w->pinned) (void)hipHostFree(w->pinned);
  w->pinned = nullptr;
  w->pinned_cap = 0;
  BSR_HIP(hipHostMalloc((void**)&w->pinned, bytes, hipHostMallocDefault));
  w->pinned_cap = bytes;
  return SNF_OK;
}

// Host-side validation of a BSR pattern: sizes, ascending columns, symmetric pattern and
// every diagonal block present.
static int validate_pattern(const snf_bsr* m, std::vector<int32_t>& rp, std::vector<int32_t>& ci,
                            hipStream_t s) {
  if (!m || m->b != kB || m->n <= 0 || m->n % kB || m->nb != m->n / kB || m->nnzb < m->nb ||
      !m->row_ptr || !m->col_idx || !m->val || m->nb > 65535)
    return SNF_EINVAL;
  rp.resize(m->nb + 1);
  ci.resize(m->nnzb);
  BSR_HIP(hipMemcpyAsync(rp.data(), m->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, s));
  BSR_HIP(hipMemcpyAsync(ci.data(), m->col_idx, ci.size() * 4, hipMemcpyDeviceToHost, s));
  BSR_HIP(hipStreamSynchronize(s));
  if (rp[0] != 0 || rp[m->nb] != m->nnzb) return SNF_EINVAL;
  std::vector<std::pair<int, int>> up, lo;
  for (int i = 0; i < m->nb; ++i) {
    if (rp[i + 1] < rp[i]) return SNF_EINVAL;
    bool diag = false;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      const int j = ci[p];
      if (j < 0 || j >= m->nb) return SNF_EINVAL;
      if (p > rp[i] && ci[p - 1] >= j) return SNF_EINVAL;
      if (j == i) diag = true;
      if (j > i) up.emplace_back(i, j);
      if (j < i) lo.emplace_back(j, i);
    }
    if (!diag) return SNF_EINVAL;
  }
  std::sort(lo.begin(), lo.end());
  if (up != lo) return SNF_EINVAL;   // up is already in (i, j) order
  return SNF_OK;
}

static int build_lookup(BsrBuf& b, int nb, int W, hipStream_t s) {
  int rc = b.bm.reserve((size_t)nb * W);
  if (rc) return rc;
  rc = b.pre.reserve((size_t)nb * W);
  if (rc) return rc;
  hipLaunchKernelGGL(bsr_bitmap_kernel, dim3(nb), dim3(64), W * sizeof(uint32_t), s, b.row_ptr.p,
                     b.col.p, W, b.bm.p, b.pre.p);
  BSR_HIP(hipGetLastError());
  return SNF_OK;
}

// exclusive scan of cnt (device, nb) into row_ptr (device, nb + 1) through pinned memory;
// returns the total
static int scan_counts(BsrWorkspace* w, const int32_t* cnt_dev, int nb, DevArr<int32_t>& row_ptr,
                       int64_t* total, hipStream_t s) {
  int rc = ensure_pinned(w, (size_t)(2 * nb + 2) * sizeof(int32_t));
  if (rc) return rc;
  int32_t* h = w->pinned;
  BSR_HIP(hipMemcpyAsync(h, cnt_dev, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  BSR_HIP(hipStreamSynchronize(s));
  int32_t* rp = h + nb + 1;
  int64_t acc = 0;
  for (int i = 0; i < nb; ++i) {
    rp[i] = (int32_t)acc;
    acc += h[i];
  }
  rp[nb] = (int32_t)acc;
  if (acc > INT32_MAX) return SNF_ENOMEM;
  rc = row_ptr.reserve(nb + 1);
  if (rc) return rc;
  BSR_HIP(hipMemcpyAsync(row_ptr.p, rp, (nb + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  *total = acc;
  return SNF_OK;
}

// One product Y = c2 A.B + c1 L + c0 I (lookup tables of A, B and L built; coefficients from
// the state) into N: candidate pattern of A.B, numeric product, truncation, compaction.  A
// square has A = B = L = X; the other products of a fixed-mu iteration (Algorithm 1's S2.X,
// the Horner levels and the last product of P_{m,m} and P_{i,j}) multiply polynomials in the
// same matrix, so A.B is symmetric and so is its pattern.  N2 (optional) receives the second
// output d2 A.B + d1 L + d0 I with the same kept blocks (P_{i,j}'s first product).  Partial sums
// land in slots [0, tiles) (product) and [tiles, tiles + nb) (kept norms); *slots = total.
// eps_i >= 0 selects the error-controlled rule (tau2 is then derived from the block-norm
// histogram of this product); eps_i < 0 keeps the fixed threshold tau2.
static int bsr_step(BsrWorkspace* w, BsrBuf& X, BsrBuf& B, BsrBuf& L, BsrBuf& N, int nb,
                    int W, double tau2, int* slots, hipEvent_t ev_a, hipEvent_t ev_b,
                    hipStream_t s, double eps_i = -1.0, double screen2 = 0.0,
                    BsrBuf* N2 = nullptr) {
  BsrBuf& P = w->P;
  int rc;
  // 1b. operand block norms for the screening (B's own when it is another matrix)
  if (screen2 > 0.0 && X.nnzb > 0) {
    if ((rc = w->nrmX.reserve(X.nnzb))) return rc;
    hipLaunchKernelGGL(bsr_block_norms_kernel, dim3((unsigned)((X.nnzb + 3) / 4)), dim3(256), 0,
                       s, X.val.p, X.nnzb, w->nrmX.p);
    BSR_HIP(hipGetLastError());
  }
  if (screen2 > 0.0 && &B != &X && B.nnzb > 0) {
    if ((rc = w->nrmY.reserve(B.nnzb))) return rc;
    hipLaunchKernelGGL(bsr_block_norms_kernel, dim3((unsigned)((B.nnzb + 3) / 4)), dim3(256), 0,
                       s, B.val.p, B.nnzb, w->nrmY.p);
    BSR_HIP(hipGetLastError());
  }
  // 2. symbolic
  if ((rc = P.bm.reserve((size_t)nb * W)) || (rc = P.pre.reserve((size_t)nb * W)) ||
      (rc = w->cnt.reserve(nb)))
    return rc;
  if ((rc = w->triples.reserve(nb))) return rc;
  hipLaunchKernelGGL(bsr_symbolic_kernel, dim3(nb), dim3(64), W * sizeof(uint32_t), s,
                     X.row_ptr.p, X.col.p, B.row_ptr.p, B.bm.p, W, B.pre.p, P.bm.p, P.pre.p,
                     w->cnt.p, w->triples.p);
  BSR_HIP(hipGetLastError());
  int64_t nnzP = 0;
  if ((rc = scan_counts(w, w->cnt.p, nb, P.row_ptr, &nnzP, s))) return rc;
  {
    // useful block triples of this product (the symbolic kernel finished: scan synced)
    std::vector<int64_t> tri(nb);
    BSR_HIP(hipMemcpy(tri.data(), w->triples.p, nb * sizeof(int64_t), hipMemcpyDeviceToHost));
    int64_t t = 0;
    for (int i = 0; i < nb; ++i) t += tri[i];
    w->last_triples = t;
  }
  if ((rc = P.col.reserve(nnzP)) || (rc = P.val.reserve((size_t)nnzP * kBB)) ||
      (rc = w->normP.reserve(nnzP)) || (rc = w->rank.reserve(nnzP)))
    return rc;
  P.nnzb = nnzP;
  hipLaunchKernelGGL(bsr_fill_cols_kernel, dim3(nb), dim3(64), 0, s, P.bm.p, P.pre.p,
                     P.row_ptr.p, W, P.col.p);
  // 3. super-tiles
  const int NT = (nb + kSup - 1) / kSup;
  if ((rc = w->flags.reserve((size_t)NT * NT))) return rc;
  const int64_t nflags = (int64_t)NT * NT;
  hipLaunchKernelGGL(bsr_tile_flags_kernel, dim3((unsigned)((nflags + 255) / 256)), dim3(256), 0,
                     s, P.bm.p, nb, W, NT, w->flags.p);
  BSR_HIP(hipGetLastError());
  if ((rc = ensure_pinned(w, (size_t)nflags + (size_t)nflags * 4 + 128))) return rc;
  uint8_t* hf = (uint8_t*)w->pinned;
  BSR_HIP(hipMemcpyAsync(hf, w->flags.p, nflags, hipMemcpyDeviceToHost, s));
  BSR_HIP(hipStreamSynchronize(s));
  int32_t* tl = (int32_t*)(hf + ((nflags + 63) / 64) * 64);
  int ntiles = 0;
  // super-tiles in squares of SQ x SQ (squares in row-major order of the upper triangle,
  // tiles row-major inside): the ~512 workgroups resident at once cover 8 bands of A rows and
  // 64 of B rows instead of one band and 512, and an XCD (workgroups go to the 8 XCDs in
  // turn) takes one column of each square, whose 8 tiles stream the same B rows
  constexpr int SQ = 8;
  for (int sa = 0; sa < NT; sa += SQ)
    for (int sb = sa; sb < NT; sb += SQ)
      for (int ti = sa; ti < sa + SQ && ti < NT; ++ti)
        for (int tj = sb; tj < sb + SQ && tj < NT; ++tj)
          if (hf[(int64_t)ti * NT + tj]) tl[ntiles++] = (int32_t)((ti << 16) | tj);
  if ((rc = w->tiles.reserve(ntiles + 1)) || (rc = w->partials.reserve((size_t)(ntiles + nb) * 4)))
    return rc;
  // pinned source: the copy runs in stream order, before any later read-back reuses it
  BSR_HIP(hipMemcpyAsync(w->tiles.p, tl, ntiles * sizeof(int32_t), hipMemcpyHostToDevice, s));
  // 4. numeric
  BsrProductArgs args;
  args.X = X.view();
  args.Y = B.view();
  args.L = L.view();
  args.P = P.view();
  args.val2 = nullptr;
  if (N2) {                              // second output, same candidate pattern
    if ((rc = w->val2.reserve((size_t)nnzP * kBB))) return rc;
    args.val2 = w->val2.p;
  }
  args.normP = w->normP.p;
  args.tiles = w->tiles.p;
  args.partials = w->partials.p;
  args.nrmX = screen2 > 0.0 ? w->nrmX.p : nullptr;
  args.nrmY = screen2 > 0.0 ? (&B == &X ? w->nrmX.p : w->nrmY.p) : nullptr;
  args.screen2 = screen2 > 0.0 ? screen2 : 0.0;
  args.nb = nb;
  args.W = W;
  if (ev_a) BSR_HIP(hipEventRecord(ev_a, s));
  if (ntiles > 0)
    hipLaunchKernelGGL(bsr_product_kernel, dim3(ntiles), dim3(512), 0, s, w->state, args);
  if (ev_b) BSR_HIP(hipEventRecord(ev_b, s));
  BSR_HIP(hipGetLastError());
  // 5. truncation (threshold from the norm histogram under error control)
  if (eps_i >= 0.0) {
    if ((rc = w->hist.reserve(kNumBins))) return rc;
    BSR_HIP(hipMemsetAsync(w->hist.p, 0, kNumBins * sizeof(uint32_t), s));
    hipLaunchKernelGGL(bsr_norm_hist_kernel, dim3(nb), dim3(64), 0, s, P.row_ptr.p, P.col.p,
                       w->normP.p, w->hist.p);
    BSR_HIP(hipGetLastError());
    BSR_HIP(hipMemcpyAsync(w->hist_host, w->hist.p, kNumBins * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    BSR_HIP(hipStreamSynchronize(s));
    tau2 = error_control_tau2(w->hist_host, eps_i);
    w->last_tau2 = tau2;
  }
  hipLaunchKernelGGL(bsr_truncate_kernel, dim3(nb), dim3(64), 0, s, P.row_ptr.p, P.col.p,
                     w->normP.p, tau2, w->rank.p, w->cnt.p, w->partials.p, ntiles);
  BSR_HIP(hipGetLastError());
  int64_t nnzN = 0;
  if ((rc = scan_counts(w, w->cnt.p, nb, N.row_ptr, &nnzN, s))) return rc;
  if ((rc = N.col.reserve(nnzN)) || (rc = N.val.reserve((size_t)nnzN * kBB))) return rc;
  N.nnzb = nnzN;
  // 6. compaction
  hipLaunchKernelGGL(bsr_compact_kernel, dim3(nb), dim3(256), 0, s, P.row_ptr.p, P.col.p, P.val.p,
                     w->rank.p, N.row_ptr.p, N.col.p, N.val.p);
  BSR_HIP(hipGetLastError());
  if (N2) {                              // the same kept blocks of the second output
    if ((rc = N2->row_ptr.reserve(nb + 1)) || (rc = N2->col.reserve(nnzN)) ||
        (rc = N2->val.reserve((size_t)nnzN * kBB)))
      return rc;
    N2->nnzb = nnzN;
    BSR_HIP(hipMemcpyAsync(N2->row_ptr.p, N.row_ptr.p, (nb + 1) * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(bsr_compact_kernel, dim3(nb), dim3(256), 0, s, P.row_ptr.p, P.col.p,
                       w->val2.p, w->rank.p, N2->row_ptr.p, N2->col.p, N2->val.p);
    BSR_HIP(hipGetLastError());
  }
  *slots = ntiles + nb;
  return SNF_OK;
}

static int copy_in(BsrWorkspace* w, const snf_bsr* F, hipStream_t s) {
  BsrBuf& Fl = w->Fl;
  int rc;
  if ((rc = Fl.row_ptr.reserve(F->nb + 1)) || (rc = Fl.col.reserve(F->nnzb))) return rc;
  BSR_HIP(hipMemcpyAsync(Fl.row_ptr.p, F->row_ptr, (F->nb + 1) * 4, hipMemcpyDeviceToDevice, s));
  BSR_HIP(hipMemcpyAsync(Fl.col.p, F->col_idx, F->nnzb * 4, hipMemcpyDeviceToDevice, s));
  Fl.nnzb = F->nnzb;
  return SNF_OK;
}

static int make_output(const BsrBuf& X, int64_t n, int nb, snf_bsr** out, hipStream_t s) {
  snf_bsr* m = (snf_bsr*)calloc(1, sizeof(snf_bsr));
  if (!m) return SNF_ENOMEM;
  m->n = n;
  m->b = kB;
  m->nb = nb;
  m->nnzb = X.nnzb;
  if (hipMalloc(&m->row_ptr, (nb + 1) * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&m->col_idx, (size_t)X.nnzb * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&m->val, (size_t)X.nnzb * kBB * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    snf_bsr_free(m);
    return SNF_ENOMEM;
  }
  BSR_HIP(hipMemcpyAsync(m->row_ptr, X.row_ptr.p, (nb + 1) * 4, hipMemcpyDeviceToDevice, s));
  BSR_HIP(hipMemcpyAsync(m->col_idx, X.col.p, X.nnzb * 4, hipMemcpyDeviceToDevice, s));
  BSR_HIP(hipMemcpyAsync(m->val, X.val.p, (size_t)X.nnzb * kBB * 4, hipMemcpyDeviceToDevice, s));
  *out = m;
  return SNF_OK;
}

static int ensure_state(BsrWorkspace* w) {
  if (!w->state) {
    BSR_HIP(hipMalloc(&w->state, sizeof(SnfState)));
    BSR_HIP(hipHostMalloc(&w->state_host, sizeof(SnfState), hipHostMallocDefault));
    for (int i = 0; i < 4; ++i) BSR_HIP(hipEventCreate(&w->ev[i]));
    BSR_HIP(hipHostMalloc(&w->hist_host, kNumBins * sizeof(uint32_t), hipHostMallocDefault));
  }
  return SNF_OK;
}

// X_0 = f_0(F) into w->X[0] (pattern of F) with its lookup tables; partial sums of
// tr X_0 and ||X_0||_F^2 in slots [0, kF0Blocks).
static int bsr_init(BsrWorkspace* w, const snf_bsr* F, int W, hipStream_t s) {
  int rc;
  const int nb = F->nb;
  if ((rc = copy_in(w, F, s))) return rc;
  if ((rc = build_lookup(w->Fl, nb, W, s))) return rc;
  BsrBuf& X = w->X[0];
  if ((rc = X.row_ptr.reserve(nb + 1)) || (rc = X.col.reserve(F->nnzb)) ||
      (rc = X.val.reserve((size_t)F->nnzb * kBB)) || (rc = w->partials.reserve(kF0Blocks * 4)))
    return rc;
  X.nnzb = F->nnzb;
  BSR_HIP(hipMemcpyAsync(X.row_ptr.p, F->row_ptr, (nb + 1) * 4, hipMemcpyDeviceToDevice, s));
  BSR_HIP(hipMemcpyAsync(X.col.p, F->col_idx, F->nnzb * 4, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(bsr_f0_kernel, dim3(kF0Blocks), dim3(256), 0, s, w->Fl.row_ptr.p,
                     w->Fl.col.p, w->Fl.bm.p, w->Fl.pre.p, F->val, W, w->state, X.val.p,
                     w->partials.p, nb);
  BSR_HIP(hipGetLastError());
  return build_lookup(X, nb, W, s);
}

}  // namespace snf

using namespace snf;

extern "C" {

int snf_bsr_copy_out(const snf_bsr* src, int32_t* row_ptr, int32_t* col_idx, float* val,
                     void* stream) {
  if (!src || !row_ptr || (src->nnzb > 0 && (!col_idx || !val))) return SNF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  BSR_HIP(hipMemcpyAsync(row_ptr, src->row_ptr, (src->nb + 1) * sizeof(int32_t),
                         hipMemcpyDeviceToDevice, s));
  if (src->nnzb > 0) {
    BSR_HIP(hipMemcpyAsync(col_idx, src->col_idx, src->nnzb * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
    BSR_HIP(hipMemcpyAsync(val, src->val, (size_t)src->nnzb * kBB * sizeof(float),
                           hipMemcpyDeviceToDevice, s));
  }
  BSR_HIP(hipStreamSynchronize(s));
  return SNF_OK;
}

void snf_bsr_free(snf_bsr* m) {
  if (!m) return;
  if (m->row_ptr) (void)hipFree(m->row_ptr);
  if (m->col_idx) (void)hipFree(m->col_idx);
  if (m->val) (void)hipFree(m->val);
  free(m);
}

namespace snf {
// Iterations the scalar recurrence of Algorithm 2 (alpha = 0 for the unscaled schemes; the
// trace scheme is predicted by that recurrence) takes until max(beta, 1 - beta-bar) <= eps.
static int predicted_iterations(snf_scheme scheme, double beta, double betabar, double eps) {
#pragma clang fp contract(off)
  for (int it = 0; it < 200; ++it) {
    const double bound = beta > 1.0 - betabar ? beta : 1.0 - betabar;
    if (bound <= eps) return it > 1 ? it : 1;
    const bool sq = sched::alg2_square(beta, betabar);
    double a = 0.0;
    if (scheme == SNF_SNF_VARMU)
      a = sq ? sched::alg2_square_alpha(beta) : sched::alg2_fold_alpha(betabar);
    if (sq) {
      beta = sched::alg2_square_map(beta, a);
      betabar = sched::alg2_square_map(betabar, a);
    } else {
      beta = sched::alg2_fold_map(beta, a);
      betabar = sched::alg2_fold_map(betabar, a);
    }
  }
  return 200;
}

// The fixed-mu schemes' scalar recurrence on the host, with the FP64 expressions the device's
// schedule uses: the alpha an iteration takes from the bounds, and the bounds of the iterate
// it produces (beta, beta-bar; for P_{i,j} also a' = 1 - beta-bar).
static double fixmu_alpha(snf_scheme scheme, const SnfState& s) {
#pragma clang fp contract(off)
  if (scheme_is_pij(scheme)) {
    if (scheme != SNF_SNF_FIXMU_PIJ) return 1.0;
    const double lo = sched::pij_alpha_side_tab(s.pij_i, s.pij_j, s.pbin[0], s.xstar, s.beta);
    const double hi =
        sched::pij_alpha_side_tab(s.pij_j, s.pij_i, s.pbin[1], 1.0 - s.xstar, s.abar);
    return lo < hi ? lo : hi;
  }
  if (scheme_pmm_m(scheme))
    return (scheme == SNF_SNF_FIXMU3 || scheme == SNF_SNF_FIXMU5)
               ? sched::pmm_alpha_tab(s.pmm_m, s.pbin[0], s.beta)
               : 1.0;
  return scheme == SNF_SNF_FIXMU ? sched::alg1_alpha(s.beta) : 1.0;
}

static void fixmu_advance(SnfState& s, double a) {
#pragma clang fp contract(off)
  if (s.pij_i) {
    const double xs = s.xstar;
    const double an = sched::pij_side_next_tab(s.pij_i, s.pij_j, s.pbin[0], xs, s.beta, a);
    const double bn = sched::pij_side_next_tab(s.pij_j, s.pij_i, s.pbin[1], 1.0 - xs, s.abar, a);
    s.beta = an;
    s.abar = bn;
    s.betabar = 1.0 - bn;
  } else if (s.pmm_m) {
    s.beta = sched::pij_eval_tab(s.pmm_m, s.pmm_m, s.pbin[0], a * (s.beta - 0.5) + 0.5);
    s.betabar = 1.0 - s.beta;
  } else {
    s.beta = sched::alg1_beta_next(s.beta, a);
    s.betabar = 1.0 - s.beta;
  }
}

// Iterations until the fixed-mu recurrence's bound (max(beta, 1 - beta-bar); for P_{i,j}
// max(a, a')) is at most eps.
static int predicted_iterations_fixmu(snf_scheme scheme, SnfState s, double eps) {
  for (int it = 0; it < 200; ++it) {
    const double bound = s.pij_i ? (s.beta > s.abar ? s.beta : s.abar)
                                 : (s.beta > 1.0 - s.betabar ? s.beta : 1.0 - s.betabar);
    if (bound <= eps) return it > 1 ? it : 1;
    fixmu_advance(s, fixmu_alpha(scheme, s));
  }
  return 200;
}

// Truncation budget of the pending step: eps g / (sqrt 2 N), g the X-space gap of the iterate
// the step produces (its bounds advanced by the step's branch and alpha).
static double error_control_eps(const SnfState* sh, double eps, int n_pred) {
#pragma clang fp contract(off)
  double b = sh->beta, bb = sh->betabar;
  if (sh->branch == SNF_BRANCH_SQUARE) {
    b = sched::alg2_square_map(b, sh->alpha);
    bb = sched::alg2_square_map(bb, sh->alpha);
  } else if (sh->branch == SNF_BRANCH_FOLD) {
    b = sched::alg2_fold_map(b, sh->alpha);
    bb = sched::alg2_fold_map(bb, sh->alpha);
  } else {                                  // the fixed-mu iterations
    SnfState t = *sh;
    fixmu_advance(t, sh->alpha);
    b = t.beta;
    bb = t.betabar;
  }
  return eps * (bb - b) / (kSqrt2 * (double)n_pred);
}
}  // namespace snf

namespace snf {
static int purify_bsr_body(const snf_bsr* F, const snf_params* params, snf_scheme scheme,
                           double trunc_tau, snf_bsr** D_out, snf_result* out,
                           snf_log_rec* log, int32_t log_cap, void* stream) {
  auto fail = [&](int rc) {
    out->status = rc;
    return rc;
  };
  if (!F || !params || !D_out || !(trunc_tau >= 0.0) || !isfinite(trunc_tau)) return fail(SNF_EINVAL);
  if ((params->flags & SNF_FLAG_TRUNC_ERROR_CONTROL) && !(trunc_tau > 0.0)) return fail(SNF_EINVAL);
  // Algorithm 2 and its unscaled forms (one product per iteration); Algorithm 1 with McWeeny
  // (its alpha = 1 form), the P_{m,m} and the P_{i,j} schemes, scaled and not (a chain of
  // products per iteration, truncation after the last; P_{i,j}'s first product has two
  // outputs over one candidate pattern).
  const bool fixmu = scheme == SNF_SNF_FIXMU || scheme == SNF_MCWEENY ||
                     scheme_pmm_m(scheme) != 0 || scheme_is_pij(scheme);
  if (scheme != SNF_SP2_TRACE && scheme != SNF_TC2_BETA && scheme != SNF_SNF_VARMU && !fixmu)
    return fail(SNF_EINVAL);
  const snf_params& p = *params;
  if (!(p.screen_tau >= 0.0) || !isfinite(p.screen_tau) || p.lowp_floor < 0.0 ||
      !(p.lowp_floor < 0.5))
    return fail(SNF_EINVAL);
  if (fixmu) {
    // the fixed-mu parameters as on the dense path (checked as for FP64, where the dense
    // path offers P_{m,m}; the block-sparse products are FP32 either way); the
    // error-control budget applies to each iteration's result, the norm screening to every
    // product of an iteration (each operand's own block norms)
    if (validate(F ? F->n : 0, params, scheme, SNF_P_FP64) != SNF_OK) return fail(SNF_EINVAL);
  } else if (!isfinite(p.lambda_min) || !isfinite(p.lambda_max) ||
             !(p.lambda_min < p.lambda_max) || !(p.tol > 0.0) || p.max_iter < 1 ||
             p.max_iter >= SNF_LOG_MAX || !isfinite(p.homo) || !isfinite(p.lumo) ||
             !(p.homo < p.lumo) || p.homo < p.lambda_min || p.lumo > p.lambda_max ||
             (scheme == SNF_SP2_TRACE && p.n_occ < 0)) {
    return fail(SNF_EINVAL);
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> rp, ci;
  int rc = validate_pattern(F, rp, ci, s);
  if (rc) return fail(rc);
  if (p.n_occ > F->n) return fail(SNF_EINVAL);
  BsrWorkspace* w = bsr_workspace();
  if (!w) return fail(SNF_EDEVICE);
  std::lock_guard<std::mutex> guard(w->mu);
  if ((rc = ensure_state(w))) return fail(rc);
  const int nb = F->nb, W = (nb + 31) / 32;

  // scalar state: FP32 products, no refinement phase, stagnation stop at the floor
  SnfState* sh = w->state_host;
  if (fixmu) {
    init_state(sh, F->n, params, scheme, SNF_P_FP32);   // gamma, beta, the P_{m,m} tables
  } else {
    memset(sh, 0, sizeof(*sh));
    sh->scheme = scheme;
    sh->max_iter = p.max_iter;
    sh->mode = SNF_P_FP32;
    sh->has_nocc = p.n_occ >= 0;
    sh->n = F->n;
    sh->n_occ = p.n_occ;
    sh->tol = p.tol;
    sh->lambda_min = p.lambda_min;
    sh->lambda_max = p.lambda_max;
    sh->mu = p.mu;
    sh->xi = p.xi;
    sh->homo = p.homo;
    sh->lumo = p.lumo;
    sh->beta = sched::alg2_f0(p.lumo, p.lambda_min, p.lambda_max);
    sh->betabar = sched::alg2_f0(p.homo, p.lambda_min, p.lambda_max);
    sh->e_hist[0] = sh->e_hist[1] = sh->e_hist[2] = INFINITY;
  }
  sh->gap_switch = 0.0;
  sh->lowp_floor = p.lowp_floor > 0.0 ? p.lowp_floor : 1e-3;
  BSR_HIP(hipMemcpyAsync(w->state, sh, sizeof(SnfState), hipMemcpyHostToDevice, s));
  BSR_HIP(hipEventRecord(w->ev[0], s));
  if ((rc = bsr_init(w, F, W, s))) return fail(rc);
  launch_schedule(w->state, w->partials.p, kF0Blocks, 1, s);
  BSR_HIP(hipGetLastError());

  const bool ec = (p.flags & SNF_FLAG_TRUNC_ERROR_CONTROL) != 0;
  const double tau2 = ec ? 0.0 : trunc_tau * trunc_tau;
  const int n_pred = !ec ? 1
                     : fixmu ? predicted_iterations_fixmu(scheme, *sh, trunc_tau)
                             : predicted_iterations(scheme, sh->beta, sh->betabar, trunc_tau);
  // the pending product's kind, branch and alpha (which product runs next; the truncation
  // budget of error control)
  BSR_HIP(hipMemcpyAsync(sh, w->state, sizeof(SnfState), hipMemcpyDeviceToHost, s));
  BSR_HIP(hipStreamSynchronize(s));
  const bool timing = (p.flags & SNF_FLAG_TIME_PRODUCTS) != 0;
  double prod_ms = 0.0, flops = 0.0;
  int cur = 0;
  std::vector<int64_t> blocks_of_iterate;   // stored blocks of X_i
  blocks_of_iterate.push_back(w->X[0].nnzb);
  // One product per pass, on the buffers the schedule names (operands ia and ib, linear term
  // ix, output io; 0 and 1 hold X, 2 and 3 an iteration's intermediates).  Only the product
  // that completes an iteration is truncated: the intermediates keep every candidate block,
  // as the oracle's mask applies to each f_i's result.
  for (int pass = 0; pass <= 8 * (p.max_iter + 1); ++pass) {
    int slots = 0;
    const bool last = sh->kind == kKindCube || sh->kind == kKindFinal ||
                      (sh->kind == kKindSquare && (sh->branch == SNF_BRANCH_SQUARE ||
                                                   sh->branch == SNF_BRANCH_FOLD));
    const double eps_i = ec ? error_control_eps(sh, trunc_tau, n_pred) : -1.0;
    BsrBuf& out = w->buf(sh->io);
    BsrBuf* out2 = sh->dual ? &w->buf(sh->io2) : nullptr;
    rc = bsr_step(w, w->buf(sh->ia), w->buf(sh->ib), w->buf(sh->ix), out, nb, W,
                  last ? tau2 : 0.0, &slots, timing ? w->ev[2] : nullptr,
                  timing ? w->ev[3] : nullptr, s, last ? eps_i : -1.0,
                  p.screen_tau * p.screen_tau, out2);
    if (rc) return fail(rc);
    launch_schedule(w->state, w->partials.p, slots, 0, s);
    BSR_HIP(hipGetLastError());
    BSR_HIP(hipMemcpyAsync(sh, w->state, sizeof(SnfState), hipMemcpyDeviceToHost, s));
    BSR_HIP(hipStreamSynchronize(s));
    if (timing) {
      float ms = 0.f;
      BSR_HIP(hipEventElapsedTime(&ms, w->ev[2], w->ev[3]));
      prod_ms += ms;
    }
    flops += 2.0 * kB * kB * kB * (double)w->last_triples;
    if (sh->stop) break;
    if ((rc = build_lookup(out, nb, W, s))) return fail(rc);
    if (out2 && (rc = build_lookup(*out2, nb, W, s))) return fail(rc);
    if (last) blocks_of_iterate.push_back(out.nnzb);
  }
  cur = sh->cur;
  // the result is the X whose idempotency was certified (the input of the last product)
  rc = make_output(w->buf(cur), F->n, nb, D_out, s);
  if (rc) return fail(rc);
  BSR_HIP(hipEventRecord(w->ev[1], s));
  BSR_HIP(hipStreamSynchronize(s));
  const int status = sh->stop ? sh->status : SNF_ENOCONV;
  out->status = status;
  out->iterations = sh->iter;
  out->products = sh->products;
  out->products_fp64 = sh->products_f64;
  out->products_lowp = sh->products_lowp;
  out->idem_err = sh->e_last;
  out->trace = sh->t1;
  out->trace_err = sh->has_nocc ? sh->t1 - (double)sh->n_occ : 0.0;
  out->alpha_last = sh->alpha;
  out->beta_last = sh->beta;
  out->betabar_last = sh->betabar;
  const int nrec = sh->nlog < SNF_LOG_MAX ? sh->nlog : SNF_LOG_MAX;
  for (int i = 0; i < nrec; ++i)
    out->branch[i] = (uint8_t)(sh->log[i].branch < 0 ? 255 : sh->log[i].branch);
  if (log && log_cap > 0) {
    const int m = std::min(nrec, (int)log_cap);
    memcpy(log, sh->log, (size_t)m * sizeof(snf_log_rec));
    // block-sparse: the spare field of record i holds the stored blocks of X_i
    for (int i = 0; i < m && i < (int)blocks_of_iterate.size(); ++i)
      log[i].reserved = (int32_t)std::min<int64_t>(blocks_of_iterate[i], INT32_MAX);
  }
  float ms = 0.f;
  BSR_HIP(hipEventElapsedTime(&ms, w->ev[0], w->ev[1]));
  out->device_ms = ms;
  out->product_ms = prod_ms;
  out->flops = flops;
  out->blocks = w->buf(cur).nnzb;
  return status;
}
}  // namespace snf

int snf_purify_bsr(const snf_bsr* F, const snf_params* params, snf_scheme scheme,
                   double trunc_tau, snf_bsr** D_out, snf_result* out, snf_log_rec* log,
                   int32_t log_cap, void* stream) {
  if (!out) return SNF_EINVAL;
  memset(out, 0, sizeof(*out));
  if (D_out) *D_out = nullptr;
  // every return path, HIP errors included, leaves its code in out->status
  const int rc = purify_bsr_body(F, params, scheme, trunc_tau, D_out, out, log, log_cap, stream);
  out->status = rc;
  return rc;
}

int snf_step_bsr(const snf_bsr* Xin, double c2, double c1, double c0, double trunc_tau,
                 double screen_tau, snf_bsr** Y_out, double* sums, double* kernel_ms,
                 void* stream) {
  if (!Y_out || !sums || !(trunc_tau >= 0.0) || !isfinite(c2) || !isfinite(c1) ||
      !isfinite(c0) || !(screen_tau >= 0.0) || !isfinite(screen_tau))
    return SNF_EINVAL;
  *Y_out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> rp, ci;
  int rc = validate_pattern(Xin, rp, ci, s);
  if (rc) return rc;
  BsrWorkspace* w = bsr_workspace();
  if (!w) return SNF_EDEVICE;
  std::lock_guard<std::mutex> guard(w->mu);
  if ((rc = ensure_state(w))) return rc;
  const int nb = Xin->nb, W = (nb + 31) / 32;
  SnfState* sh = w->state_host;
  memset(sh, 0, sizeof(*sh));
  sh->c2 = c2;
  sh->c1 = c1;
  sh->c0 = c0;
  sh->want_e = 1;
  BSR_HIP(hipMemcpyAsync(w->state, sh, sizeof(SnfState), hipMemcpyHostToDevice, s));
  BsrBuf& X = w->X[0];
  if ((rc = X.row_ptr.reserve(nb + 1)) || (rc = X.col.reserve(Xin->nnzb)) ||
      (rc = X.val.reserve((size_t)Xin->nnzb * kBB)))
    return rc;
  X.nnzb = Xin->nnzb;
  BSR_HIP(hipMemcpyAsync(X.row_ptr.p, Xin->row_ptr, (nb + 1) * 4, hipMemcpyDeviceToDevice, s));
  BSR_HIP(hipMemcpyAsync(X.col.p, Xin->col_idx, Xin->nnzb * 4, hipMemcpyDeviceToDevice, s));
  if ((rc = build_lookup(X, nb, W, s))) return rc;
  hipLaunchKernelGGL(bsr_sym_copy_kernel, dim3(kF0Blocks), dim3(256), 0, s, X.row_ptr.p, X.col.p,
                     X.bm.p, X.pre.p, W, Xin->val, X.val.p, nb);
  BSR_HIP(hipGetLastError());
  int slots = 0;
  if ((rc = bsr_step(w, X, X, X, w->X[1], nb, W, trunc_tau * trunc_tau, &slots, w->ev[2],
                     w->ev[3], s, -1.0, screen_tau * screen_tau)))
    return rc;
  if ((rc = ensure_pinned(w, 64)) || (rc = w->sums.reserve(4))) return rc;
  launch_sum_partials(w->partials.p, slots, w->sums.p, s);
  BSR_HIP(hipGetLastError());
  BSR_HIP(hipMemcpyAsync(w->pinned, w->sums.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  rc = make_output(w->X[1], Xin->n, nb, Y_out, s);
  BSR_HIP(hipStreamSynchronize(s));
  if (rc) return rc;
  const double* hs = (const double*)w->pinned;
  sums[0] = hs[0];
  sums[1] = hs[1];
  sums[2] = hs[2];
  if (kernel_ms) {
    float ms = 0.f;
    BSR_HIP(hipEventElapsedTime(&ms, w->ev[2], w->ev[3]));
    *kernel_ms = ms;
  }
  return SNF_OK;
}

}  // extern "C"
