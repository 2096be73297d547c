// Dense kernels of libsnf for gfx950 (MI355X, CDNA4).
//
//  * f0_kernel        -- X_0 = f_0(F) (Algorithm 1 or 2 initial map) into a zero-padded
//                        n_pad x n_pad buffer, symmetric by construction (upper triangle of F
//                        read, LDS-transposed for the lower half), plus per-block partial sums
//                        of tr X_0 and ||X_0||_F^2 and the low-precision operand copy.
//  * product kernels  -- P = A.B for symmetric A, B on MFMA (f64 16x16x4, f32 16x16x4,
//                        bf16 16x16x32 with f32 accumulation), LDS double-buffered 128x128
//                        output tiles, only the upper triangle of tiles (P is symmetric) with
//                        the mirror written by the same workgroup; fused epilogue
//                        Y = c2 P + c1 X + c0 I and FP64 partial sums of ||P - X||_F^2,
//                        tr Y, ||Y||_F^2 per tile.
//  * schedule_kernel  -- one workgroup: fixed-order reduction of the per-tile partials and the
//                        scalar state machine (branch, alpha, beta, beta-bar, stopping).
//  * copy kernels     -- padded <-> caller layout.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "schedule_math.h"
#include "snf_internal.h"

namespace snf {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
  // round-to-nearest-even truncation of an IEEE binary32 to bfloat16 (NaN kept quiet)
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// ---------------------------------------------------------------------------------------
// Wave / block reductions in a fixed order (deterministic).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum three values over a 256-thread block; result valid in thread 0.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* lds12) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    lds12[w * 3 + 0] = a;
    lds12[w * 3 + 1] = b;
    lds12[w * 3 + 2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = ((lds12[0] + lds12[3]) + lds12[6]) + lds12[9];
    b = ((lds12[1] + lds12[4]) + lds12[7]) + lds12[10];
    c = ((lds12[2] + lds12[5]) + lds12[8]) + lds12[11];
  }
}

// ---------------------------------------------------------------------------------------
// f0: X_0 = f_0(F)
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void f0_kernel(const double* __restrict__ F, int64_t n,
                                                 int64_t ld, int64_t np,
                                                 const SnfState* __restrict__ st,
                                                 const Buffers* __restrict__ bufs,
                                                 int lowp_kind, double* __restrict__ partials) {
  __shared__ double tile[32][33];
  __shared__ double red[12];
  const int alg1 = (st->scheme == SNF_MCWEENY || st->scheme == SNF_SNF_FIXMU);
  const double lmin = st->lambda_min, lmax = st->lambda_max, mu = st->mu, gamma = st->gamma;
  double* X = bufs->x[st->cur];
  void* LP = bufs->lp[st->cur];
  const int64_t nt = np / 32;
  const int64_t ntiles = nt * nt;
  double t1 = 0.0, t2 = 0.0;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t bi = t / nt, bj = t % nt;
    const int64_t si = bi < bj ? bi : bj, sj = bi < bj ? bj : bi;  // source tile (upper)
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int64_t gr = si * 32 + r, gc = sj * 32 + tx;
      tile[r][tx] = (gr < n && gc < n) ? F[gr * ld + gc] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int64_t gr = bi * 32 + r, gc = bj * 32 + tx;
      const double v = (gr <= gc) ? tile[r][tx] : tile[tx][r];
      double x = 0.0;
      if (gr < n && gc < n) {
        const bool d = (gr == gc);
        if (alg1) {
          x = ((d ? mu : 0.0) - v) / gamma + (d ? 0.5 : 0.0);
        } else {
          x = ((d ? lmax : 0.0) - v) / (lmax - lmin);
        }
        if (d) t1 += x;
        t2 += x * x;
      }
      X[gr * np + gc] = x;
      if (lowp_kind == kPrecF32) {
        ((float*)LP)[gr * np + gc] = (float)x;
      } else if (lowp_kind == kPrecBF16) {
        ((unsigned short*)LP)[gr * np + gc] = f32_to_bf16_rne((float)x);
      }
    }
  }
  double e0 = 0.0;
  block_sum3(e0, t1, t2, red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = 0.0;
    partials[blockIdx.x * 4 + 1] = t1;
    partials[blockIdx.x * 4 + 2] = t2;
    partials[blockIdx.x * 4 + 3] = 0.0;
  }
}

void launch_f0(const double* F, int64_t n, int64_t ld, int64_t np, SnfState* st,
               const Buffers* bufs_dev, int lowp_kind, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(f0_kernel, dim3(kF0Blocks), dim3(256), 0, s, F, n, ld, np, st, bufs_dev,
                     lowp_kind, partials);
}

// ---------------------------------------------------------------------------------------
// Tile enumeration: upper triangle of 128x128 tiles (bi <= bj) or the full grid, with the
// workgroup id remapped so that each XCD (workgroups are dealt round-robin to the 8 XCDs)
// works on a contiguous stretch of the tile list, which shares operand panels in its L2.
// ---------------------------------------------------------------------------------------
int num_product_tiles(int64_t np, int sym) {
  const int64_t nt = np / kTile;
  return (int)(sym ? nt * (nt + 1) / 2 : nt * nt);
}

__device__ __forceinline__ int xcd_remap(int w, int total) {
  const int xcd = w & 7, slot = w >> 3;
  const int base = total >> 3, rem = total & 7;
  return xcd * base + (xcd < rem ? xcd : rem) + slot;
}

__device__ __forceinline__ void tile_coords(int t, int nt, int sym, int& bi, int& bj) {
  if (!sym) {
    bi = t / nt;
    bj = t % nt;
    return;
  }
  // row-major over the upper triangle: row r holds nt - r tiles
  int r = 0, rem = t;
  while (rem >= nt - r) {
    rem -= nt - r;
    ++r;
  }
  bi = r;
  bj = r + rem;
}

// ---------------------------------------------------------------------------------------
// Product kernel, f64 / f32 MFMA 16x16x4.
//   LDS tiles hold 'k-rows' of both operands: sA[k][i] = A[k0+k][i0+i] and
//   sB[k][j] = B[k0+k][j0+j]; A[i][k] = A[k][i] because A is symmetric, so both panels are
//   read with contiguous, coalesced rows.  MFMA operand of lane l: row/col (l % 16), k (l / 16).
// ---------------------------------------------------------------------------------------
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef dbl4 acc_t;
  static constexpr int kBK = 16;   // k-depth per stage (128 B per LDS row)
  static constexpr int kPad = 16;  // row stride 144 doubles = 1152 B
  __device__ static __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef flt4 acc_t;
  static constexpr int kBK = 32;
  static constexpr int kPad = 16;  // row stride 144 floats = 576 B
  __device__ static __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Shared epilogue over the 64x64 wave tile held as acc[4][4] (MFMA 16x16 blocks).
// Accumulator layout of lane l, register v: column l % 16 and row
//   4 (l / 16) + v   for the f32 and bf16 MFMAs (ROWS_INTERLEAVED = false),
//   (l / 16) + 4 v   for the f64 MFMA          (ROWS_INTERLEAVED = true).
template <bool ROWS_INTERLEAVED, typename AccT>
__device__ __forceinline__ void epilogue(const AccT (&acc)[4][4], int gi0, int gj0, int sym,
                                         int diag, int64_t n, int64_t np,
                                         const double* __restrict__ Xt,
                                         double* __restrict__ Y, void* __restrict__ LPY,
                                         int lowp_kind, double c2, double c1, double c0,
                                         int want_e, double& e2, double& t1, double& t2) {
  const int lane = threadIdx.x & 63;
  const int rsub = ROWS_INTERLEAVED ? (lane >> 4) : 4 * (lane >> 4), csub = lane & 15;
  const int rstep = ROWS_INTERLEAVED ? 4 : 1;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t c = gj0 + q * 16 + csub;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = gi0 + m * 16 + rsub + v * rstep;
        // In symmetric mode a diagonal tile keeps its upper half and mirrors it, so the
        // result is exactly symmetric; every off-diagonal entry then stands for two.
        if (diag && sym && r > c) continue;
        const bool mirror = sym && r != c;
        const double w = mirror ? 2.0 : 1.0;
        const double p = (double)acc[m][q][v];
        const double x = Xt[r * np + c];
        if (want_e) {
          const double d = p - x;
          e2 += w * (d * d);
        }
        double y = c2 * p + c1 * x + (r == c ? c0 : 0.0);
        if (r >= n || c >= n) y = 0.0;
        if (r == c) t1 += y;
        t2 += w * (y * y);
        Y[r * np + c] = y;
        if (mirror) Y[c * np + r] = y;
        if (lowp_kind == kPrecF32) {
          const float yf = (float)y;
          ((float*)LPY)[r * np + c] = yf;
          if (mirror) ((float*)LPY)[c * np + r] = yf;
        } else if (lowp_kind == kPrecBF16) {
          const unsigned short yb = f32_to_bf16_rne((float)y);
          ((unsigned short*)LPY)[r * np + c] = yb;
          if (mirror) ((unsigned short*)LPY)[c * np + r] = yb;
        }
      }
    }
  }
}

__device__ __forceinline__ void write_partials(double e2, double t1, double t2,
                                               double* partials, int tile) {
  __shared__ double red[12];
  block_sum3(e2, t1, t2, red);
  if (threadIdx.x == 0) {
    partials[tile * 4 + 0] = e2;
    partials[tile * 4 + 1] = t1;
    partials[tile * 4 + 2] = t2;
    partials[tile * 4 + 3] = 0.0;
  }
}

template <typename T, int PREC>
__global__ __launch_bounds__(256) void product_kernel(const SnfState* __restrict__ st,
                                                      const Buffers* __restrict__ bufs,
                                                      int64_t np, int64_t n,
                                                      double* __restrict__ partials,
                                                      int sym) {
  if (st->stop || st->prec != PREC) return;
  typedef Mfma<T> M;
  constexpr int BK = M::kBK, LDS_W = kTile + M::kPad;
  constexpr int VE = 16 / sizeof(T);          // elements per 16-byte vector
  constexpr int VPR = kTile / VE;             // vectors per LDS row
  constexpr int RPP = kThreads / VPR;         // rows per load pass
  constexpr int PASSES = BK / RPP;
  __shared__ __attribute__((aligned(16))) T sA[2][BK][LDS_W];
  __shared__ __attribute__((aligned(16))) T sB[2][BK][LDS_W];

  const int ia = st->ia, ib = st->ib, ixx = st->ix, io = st->io;
  const T* A = (PREC == kPrecF64) ? (const T*)bufs->x[ia] : (const T*)bufs->lp[ia];
  const T* B = (PREC == kPrecF64) ? (const T*)bufs->x[ib] : (const T*)bufs->lp[ib];
  const double* Xt = bufs->x[ixx];
  double* Y = bufs->x[io];
  void* LPY = bufs->lp[io];
  const int lowp_kind = st->write_lowp ? (st->mode == SNF_P_BF16_REF64 ? kPrecBF16 : kPrecF32) : -1;
  const double c2 = st->c2, c1 = st->c1, c0 = st->c0;
  const int want_e = st->want_e;

  const int nt = (int)(np / kTile);
  const int total = gridDim.x;
  const int tile = xcd_remap(blockIdx.x, total);
  int bi, bj;
  tile_coords(tile, nt, sym, bi, bj);
  const int diag = (bi == bj);
  const int64_t i0 = (int64_t)bi * kTile, j0 = (int64_t)bj * kTile;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int lrow = tid / VPR, lvec = tid % VPR;

  typename M::acc_t acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[m][q] = typename M::acc_t{0, 0, 0, 0};

  u32x4 ra[PASSES], rb[PASSES];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const int64_t k = k0 + p * RPP + lrow;
      ra[p] = *(const u32x4*)(A + k * np + i0 + lvec * VE);
      rb[p] = *(const u32x4*)(B + k * np + j0 + lvec * VE);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      *(u32x4*)(&sA[buf][p * RPP + lrow][lvec * VE]) = ra[p];
      *(u32x4*)(&sB[buf][p * RPP + lrow][lvec * VE]) = rb[p];
    }
  };

  const int KT = (int)(np / BK);
  gload(0);
  lstore(0);
  __syncthreads();
  const int fr = lane & 15, fk = lane >> 4;
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) gload((int64_t)(kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[4], b[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) a[m] = sA[buf][kk + fk][wr * 64 + m * 16 + fr];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = sB[buf][kk + fk][wc * 64 + q * 16 + fr];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[m][q] = M::mma(a[m], b[q], acc[m][q]);
    }
    if (kt + 1 < KT) lstore(buf ^ 1);
    __syncthreads();
  }

  double e2 = 0.0, t1 = 0.0, t2 = 0.0;
  epilogue<PREC == kPrecF64>(acc, (int)(i0 + wr * 64), (int)(j0 + wc * 64), sym, diag, n, np,
                             Xt, Y, LPY, lowp_kind, c2, c1, c0, want_e, e2, t1, t2);
  write_partials(e2, t1, t2, partials, tile);
}

// ---------------------------------------------------------------------------------------
// Product kernel, bf16 MFMA 16x16x32 with f32 accumulation.
//   Here the LDS tiles are 'row panels' with k contiguous: sA[i][k] = A[i0+i][k0+k] and
//   sB[j][k] = B[j0+j][k0+k] (B[k][j] = B[j][k] by symmetry), because a lane's MFMA operand
//   is 8 consecutive k values of one row / column: lane l holds row (l % 16),
//   k = 8 (l / 16) .. 8 (l / 16) + 7.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void product_bf16_kernel(const SnfState* __restrict__ st,
                                                           const Buffers* __restrict__ bufs,
                                                           int64_t np, int64_t n,
                                                           double* __restrict__ partials,
                                                           int sym) {
  if (st->stop || st->prec != kPrecBF16) return;
  constexpr int BK = 64;                 // bf16 per LDS row per stage = 128 B
  constexpr int LDS_W = BK + 8;          // row stride 144 B
  constexpr int VPR = BK / 8;            // 16-byte vectors per row = 8
  constexpr int RPP = kThreads / VPR;    // 32 rows per pass
  constexpr int PASSES = kTile / RPP;    // 4
  __shared__ __attribute__((aligned(16))) unsigned short sA[2][kTile][LDS_W];
  __shared__ __attribute__((aligned(16))) unsigned short sB[2][kTile][LDS_W];

  const unsigned short* A = (const unsigned short*)bufs->lp[st->ia];
  const unsigned short* B = (const unsigned short*)bufs->lp[st->ib];
  const double* Xt = bufs->x[st->ix];
  double* Y = bufs->x[st->io];
  void* LPY = bufs->lp[st->io];
  const int lowp_kind = st->write_lowp ? kPrecBF16 : -1;
  const double c2 = st->c2, c1 = st->c1, c0 = st->c0;
  const int want_e = st->want_e;

  const int nt = (int)(np / kTile);
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  int bi, bj;
  tile_coords(tile, nt, sym, bi, bj);
  const int diag = (bi == bj);
  const int64_t i0 = (int64_t)bi * kTile, j0 = (int64_t)bj * kTile;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int lrow = tid / VPR, lvec = tid % VPR;

  flt4 acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[m][q] = flt4{0.f, 0.f, 0.f, 0.f};

  u32x4 ra[PASSES], rb[PASSES];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const int64_t r = p * RPP + lrow;
      ra[p] = *(const u32x4*)(A + (i0 + r) * np + k0 + lvec * 8);
      rb[p] = *(const u32x4*)(B + (j0 + r) * np + k0 + lvec * 8);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      *(u32x4*)(&sA[buf][p * RPP + lrow][lvec * 8]) = ra[p];
      *(u32x4*)(&sB[buf][p * RPP + lrow][lvec * 8]) = rb[p];
    }
  };

  const int KT = (int)(np / BK);
  gload(0);
  lstore(0);
  __syncthreads();
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) gload((int64_t)(kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      bf16x8 a[4], b[4];
#pragma unroll
      for (int m = 0; m < 4; ++m)
        a[m] = *(const bf16x8*)(&sA[buf][wr * 64 + m * 16 + fr][kk + fk]);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        b[q] = *(const bf16x8*)(&sB[buf][wc * 64 + q * 16 + fr][kk + fk]);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[q], acc[m][q], 0, 0, 0);
    }
    if (kt + 1 < KT) lstore(buf ^ 1);
    __syncthreads();
  }

  double e2 = 0.0, t1 = 0.0, t2 = 0.0;
  epilogue<false>(acc, (int)(i0 + wr * 64), (int)(j0 + wc * 64), sym, diag, n, np, Xt, Y,
                  LPY, lowp_kind, c2, c1, c0, want_e, e2, t1, t2);
  write_partials(e2, t1, t2, partials, tile);
}

void launch_product(int prec, SnfState* st, const Buffers* bufs_dev, int64_t np, int64_t n,
                    double* partials, int sym, hipStream_t s) {
  const int tiles = num_product_tiles(np, sym);
  if (prec == kPrecF64) {
    hipLaunchKernelGGL((product_kernel<double, kPrecF64>), dim3(tiles), dim3(kThreads), 0, s,
                       st, bufs_dev, np, n, partials, sym);
  } else if (prec == kPrecF32) {
    hipLaunchKernelGGL((product_kernel<float, kPrecF32>), dim3(tiles), dim3(kThreads), 0, s,
                       st, bufs_dev, np, n, partials, sym);
  } else {
    hipLaunchKernelGGL(product_bf16_kernel, dim3(tiles), dim3(kThreads), 0, s, st, bufs_dev,
                       np, n, partials, sym);
  }
}

// ---------------------------------------------------------------------------------------
// Schedule: reduce the partials in a fixed order, then advance the scalar state.
// ---------------------------------------------------------------------------------------
__device__ void decide(SnfState* s) {
#pragma clang fp contract(off)
  // precision phase (only for the mixed-precision modes)
  if (s->mode != SNF_P_FP64) {
    if (s->phase == kPhaseHigh && (s->betabar - s->beta) >= s->gap_switch) s->phase = kPhaseLow;
    if (s->phase == kPhaseLow && s->mode != SNF_P_FP32) {
      const double bound = s->beta > 1.0 - s->betabar ? s->beta : 1.0 - s->betabar;
      if (bound <= s->lowp_floor) s->phase = kPhaseRefine;
    }
  }
  s->prec = (s->phase == kPhaseLow) ? (s->mode == SNF_P_BF16_REF64 ? kPrecBF16 : kPrecF32)
                                    : kPrecF64;
  s->write_lowp = (s->mode != SNF_P_FP64 && s->phase != kPhaseRefine) ? 1 : 0;

  int scheme = s->scheme;
  if (s->phase == kPhaseRefine) scheme = s->has_nocc ? SNF_SP2_TRACE : SNF_MCWEENY;

  double a = 0.0;
  int br;
  if (scheme == SNF_SP2_TRACE) {
    br = sched::trace_square(s->t1, s->t2, (double)s->n_occ) ? SNF_BRANCH_SQUARE
                                                             : SNF_BRANCH_FOLD;
  } else if (scheme == SNF_TC2_BETA || scheme == SNF_SNF_VARMU) {
    const bool sq = sched::alg2_square(s->beta, s->betabar);
    br = sq ? SNF_BRANCH_SQUARE : SNF_BRANCH_FOLD;
    if (scheme == SNF_SNF_VARMU)
      a = sq ? sched::alg2_square_alpha(s->beta) : sched::alg2_fold_alpha(s->betabar);
  } else {
    br = SNF_BRANCH_P11;
    a = (scheme == SNF_SNF_FIXMU) ? sched::alg1_alpha(s->beta) : 1.0;
  }
  s->branch = br;
  s->alpha = a;
  if (br == SNF_BRANCH_SQUARE) {          // ((1+a) X - a I)^2 = (1+a)^2 P - 2a(1+a) X + a^2 I
    s->c2 = (1.0 + a) * (1.0 + a);
    s->c1 = -2.0 * a * (1.0 + a);
    s->c0 = a * a;
  } else if (br == SNF_BRANCH_FOLD) {     // 2(1+a) X - (1+a)^2 P
    s->c2 = -((1.0 + a) * (1.0 + a));
    s->c1 = 2.0 * (1.0 + a);
    s->c0 = 0.0;
  } else {                                // S2 = Xs^2 = a^2 P + 2 a c X + c^2 I, c = (1-a)/2
    const double c = 0.5 * (1.0 - a);
    s->c2 = a * a;
    s->c1 = 2.0 * a * c;
    s->c0 = c * c;
  }
  s->kind = kKindSquare;
  s->want_e = 1;
  s->ia = s->ib = s->ix = s->cur;
  s->io = (br == SNF_BRANCH_P11) ? 2 : 1 - s->cur;
}

__device__ void advance_beta(SnfState* s, int br, double a) {
#pragma clang fp contract(off)
  if (br == SNF_BRANCH_SQUARE) {
    s->beta = sched::alg2_square_map(s->beta, a);
    s->betabar = sched::alg2_square_map(s->betabar, a);
  } else if (br == SNF_BRANCH_FOLD) {
    s->beta = sched::alg2_fold_map(s->beta, a);
    s->betabar = sched::alg2_fold_map(s->betabar, a);
  } else {
    s->beta = sched::alg1_beta_next(s->beta, a);
    s->betabar = 1.0 - s->beta;
  }
}

__device__ void finish(SnfState* s, int status) {
  if ((status == SNF_OK || status == SNF_OK_FLOOR) && s->has_nocc) {
    const double err = s->t1 - (double)s->n_occ;
    if (fabs(err) >= 0.5) status = SNF_EMIXED;
  }
  s->status = status;
  s->stop = 1;
}

__global__ __launch_bounds__(kReduceThreads) void schedule_kernel(SnfState* __restrict__ s,
                                                                  const double* __restrict__ partials,
                                                                  int count, int init) {
  if (s->stop) return;
  __shared__ double red[12];
  double e2 = 0.0, t1 = 0.0, t2 = 0.0;
  for (int i = threadIdx.x; i < count; i += kReduceThreads) {
    e2 += partials[i * 4 + 0];
    t1 += partials[i * 4 + 1];
    t2 += partials[i * 4 + 2];
  }
  block_sum3(e2, t1, t2, red);
  if (threadIdx.x != 0) return;

  if (init) {
    s->t1 = t1;
    s->t2 = t2;
    decide(s);
    return;
  }
  if (s->kind == kKindSquare) {
    const double e = sqrt(e2);
    s->products += 1;
    if (s->prec == kPrecF64) s->products_f64 += 1; else s->products_lowp += 1;
    s->e_last = e;
    const int it = s->iter;
    snf_log_rec* rec = &s->log[it < SNF_LOG_MAX ? it : SNF_LOG_MAX - 1];
    rec->i = it;
    rec->branch = s->branch;
    rec->precision = s->prec;
    rec->reserved = s->phase;
    rec->alpha = s->alpha;
    rec->beta = s->beta;
    rec->betabar = s->betabar;
    rec->e = e;
    rec->t1 = s->t1;
    rec->t2 = s->t2;
    s->nlog = it + 1;
    s->e_hist[2] = s->e_hist[1];
    s->e_hist[1] = s->e_hist[0];
    s->e_hist[0] = e;
    if (!isfinite(e)) { rec->branch = -1; finish(s, SNF_ENONFINITE); return; }
    if (e <= s->tol) { rec->branch = -1; finish(s, SNF_OK); return; }
    if (s->phase == kPhaseLow && s->mode == SNF_P_FP32 && it >= 2) {
      // floor of the FP32-only mode: stop once the predicted error is below the floor
      // parameter and the measured idempotency stopped shrinking
      const double bound = s->beta > 1.0 - s->betabar ? s->beta : 1.0 - s->betabar;
      if (bound <= s->lowp_floor && e > 0.5 * s->e_hist[2]) {
        rec->branch = -1;
        finish(s, SNF_OK_FLOOR);
        return;
      }
    }
    if (it >= s->max_iter) { rec->branch = -1; finish(s, SNF_ENOCONV); return; }
    if (s->branch == SNF_BRANCH_P11) {
      // second product of Algorithm 1: R = S2.X; X_new = (3 - 2c) S2 - 2 a R
      const double a = s->alpha, c = 0.5 * (1.0 - a);
      s->kind = kKindCube;
      s->want_e = 0;
      s->c2 = -2.0 * a;
      s->c1 = 3.0 - 2.0 * c;
      s->c0 = 0.0;
      s->ia = 2;            // S2
      s->ib = s->cur;       // X
      s->ix = 2;
      s->io = 1 - s->cur;
      return;
    }
    advance_beta(s, s->branch, s->alpha);
    s->iter = it + 1;
    s->cur = s->io;
    s->t1 = t1;
    s->t2 = t2;
    decide(s);
  } else {
    s->products += 1;
    if (s->prec == kPrecF64) s->products_f64 += 1; else s->products_lowp += 1;
    advance_beta(s, SNF_BRANCH_P11, s->alpha);
    s->iter += 1;
    s->cur = s->io;
    s->t1 = t1;
    s->t2 = t2;
    decide(s);
  }
}

void launch_schedule(SnfState* st, const double* partials, int count, int init,
                     hipStream_t s) {
  hipLaunchKernelGGL(schedule_kernel, dim3(1), dim3(kReduceThreads), 0, s, st, partials,
                     count, init);
}

// ---------------------------------------------------------------------------------------
// Copies
// ---------------------------------------------------------------------------------------
__global__ void copy_out_kernel(const SnfState* __restrict__ st, const Buffers* __restrict__ bufs,
                                int64_t n, int64_t np, double* __restrict__ D, int64_t ld) {
  const double* X = bufs->x[st->cur];
  const int64_t total = n * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / n, c = t % n;
    D[r * ld + c] = X[r * np + c];
  }
}

void launch_copy_out(const SnfState* st, const Buffers* bufs_dev, int64_t n, int64_t np,
                     double* D, int64_t ld, hipStream_t s) {
  hipLaunchKernelGGL(copy_out_kernel, dim3(kF0Blocks), dim3(256), 0, s, st, bufs_dev, n, np, D,
                     ld);
}

__global__ void pad_copy_kernel(const double* __restrict__ src, int64_t n, int64_t ld,
                                double* __restrict__ dst, int64_t np, void* __restrict__ lp,
                                int lowp_kind) {
  const int64_t total = np * np;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / np, c = t % np;
    const double v = (r < n && c < n) ? src[r * ld + c] : 0.0;
    dst[t] = v;
    if (lowp_kind == kPrecF32) ((float*)lp)[t] = (float)v;
    else if (lowp_kind == kPrecBF16) ((unsigned short*)lp)[t] = f32_to_bf16_rne((float)v);
  }
}

void launch_pad_copy(const double* src, int64_t n, int64_t ld, double* dst, int64_t np,
                     void* lp_dst, int lowp_kind, hipStream_t s) {
  hipLaunchKernelGGL(pad_copy_kernel, dim3(kF0Blocks), dim3(256), 0, s, src, n, ld, dst, np,
                     lp_dst, lowp_kind);
}

__global__ void unpad_copy_kernel(const double* __restrict__ src, int64_t np, int64_t n,
                                  double* __restrict__ dst, int64_t ld) {
  const int64_t total = n * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / n, c = t % n;
    dst[r * ld + c] = src[r * np + c];
  }
}

void launch_unpad_copy(const double* src, int64_t np, int64_t n, double* dst, int64_t ld,
                       hipStream_t s) {
  hipLaunchKernelGGL(unpad_copy_kernel, dim3(kF0Blocks), dim3(256), 0, s, src, np, n, dst, ld);
}

__global__ void sum_partials_kernel(const double* __restrict__ partials, int count,
                                    double* __restrict__ out3) {
  __shared__ double red[12];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < count; i += kReduceThreads) {
    a += partials[i * 4 + 0];
    b += partials[i * 4 + 1];
    c += partials[i * 4 + 2];
  }
  block_sum3(a, b, c, red);
  if (threadIdx.x == 0) {
    out3[0] = a;
    out3[1] = b;
    out3[2] = c;
  }
}

void launch_sum_partials(const double* partials, int count, double* out3, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kReduceThreads), 0, s, partials, count,
                     out3);
}

}  // namespace snf
