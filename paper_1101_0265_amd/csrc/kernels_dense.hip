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
//                        The FP64 variant with a second epilogue output serves the first
//                        product of a P_{i,j} iteration.
//  * small orders     -- 32x32 output tiles with the k range split over the four waves of a
//                        workgroup (no split fix-up), and, at the smallest orders, the whole
//                        step loop of a solve in one cooperative launch.
//  * schedule_kernel  -- one workgroup: fixed-order reduction of the per-tile partials and the
//                        scalar state machine (branch, alpha, beta, beta-bar, stopping).
//  * copy kernels     -- padded <-> caller layout.
//  * grouped kernels  -- the serving loop's step over many requests in one launch.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_cooperative_groups.h>

#include "schedule_math.h"
#include "snf_internal.h"

namespace snf {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 16-byte load through a global-address-space pointer, so the compiler emits global_load
// (counted by vmcnt only) instead of flat_load, whose completion is also tracked by lgkmcnt
// and would make every LDS-read wait of the main loop wait for the operand prefetch too.
template <typename T>
__device__ __forceinline__ u32x4 gload16(const T* p) {
  return *(const __attribute__((address_space(1))) u32x4*)(p);
}

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

// Sum three values over the block (up to 8 waves), in wave order; result valid in thread 0.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* lds24) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    lds24[w * 3 + 0] = a;
    lds24[w * 3 + 1] = b;
    lds24[w * 3 + 2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    double sa = lds24[0], sb = lds24[1], sc = lds24[2];
    for (int i = 1; i < nw; ++i) {
      sa += lds24[3 * i + 0];
      sb += lds24[3 * i + 1];
      sc += lds24[3 * i + 2];
    }
    a = sa;
    b = sb;
    c = sc;
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
  __shared__ double red[24];
  const int alg1 = (st->scheme == SNF_MCWEENY || st->scheme == SNF_SNF_FIXMU || st->pmm_m ||
                    st->pij_i);
  const double lmin = st->lambda_min, lmax = st->lambda_max, mu = st->mu, gamma = st->gamma;
  const double xs = st->xstar;
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
          x = ((d ? mu : 0.0) - v) / gamma + (d ? xs : 0.0);
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

__device__ __forceinline__ int num_product_tiles_dev(int64_t np) {
  const int64_t nt = np / kTile;
  return (int)(nt * (nt + 1) / 2);
}

__device__ __forceinline__ int xcd_remap(int w, int total) {
  const int xcd = w & 7, slot = w >> 3;
  const int base = total >> 3, rem = total & 7;
  return xcd * base + (xcd < rem ? xcd : rem) + slot;
}

// Order of the upper-triangle tiles: the triangle is cut into blocks of kOrderG x kOrderG
// tiles; the off-diagonal blocks come first (row-major over the blocks, row-major inside a
// block), then the diagonal blocks (their upper triangles, row-major).  A full off-diagonal
// block is 64 tiles, what one XCD runs at once (32 CUs x 2 workgroups), and needs 16 operand
// panels (tile (i, j) reads row panels i and j, by symmetry).  Summed over the XCDs and
// their waves of 64, the row-major order of the whole triangle touches 1.4x as many panels
// at n = 4096 and 2.7x at n = 8192.
constexpr int kOrderG = 8;

__device__ __forceinline__ void tile_coords(int t, int nt, int sym, int& bi, int& bj) {
  if (!sym) {
    bi = t / nt;
    bj = t % nt;
    return;
  }
  const int G = kOrderG;
  const int nb = (nt + G - 1) / G;
  // off-diagonal blocks: block row P holds G * (nt - (P + 1) G) tiles (only the last block
  // row and column can be partial, and the last block row has no off-diagonal block)
  int rem = t;
  for (int P = 0; P + 1 < nb; ++P) {
    const int right = nt - (P + 1) * G;
    const int cnt = G * right;
    if (rem < cnt) {
      const int q = rem / (G * G);               // full blocks to the left in this row
      const int Q = P + 1 + q;
      const int hq = min(G, nt - Q * G);
      const int rr = rem - q * G * G;
      bi = P * G + rr / hq;
      bj = Q * G + rr % hq;
      return;
    }
    rem -= cnt;
  }
  // diagonal blocks: block P of h = min(G, nt - P G) tiles a side holds h (h + 1) / 2
  for (int P = 0; P < nb; ++P) {
    const int h = min(G, nt - P * G);
    const int cnt = h * (h + 1) / 2;
    if (rem < cnt || P + 1 == nb) {
      int r = 0;
      while (rem >= h - r) {
        rem -= h - r;
        ++r;
      }
      bi = P * G + r;
      bj = P * G + r + rem;
      return;
    }
    rem -= cnt;
  }
}

// ---------------------------------------------------------------------------------------
// MFMA wrappers, the shared epilogue, slices
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
struct EpiArgs {
  const double* Xt;  // linear term X (FP64)
  double* Y;         // output (FP64)
  void* LPY;         // low-precision copy of the output, or unused
  double* Y2;        // second output d2 P + d1 X + d0 I (FP64), or null
  int lowp_kind;     // kPrecF32 / kPrecBF16 / -1
  int want_e;
  double c2, c1, c0;
  double d2, d1, d0;
};

__device__ __forceinline__ EpiArgs epi_args(const SnfState* st, const Buffers* bufs) {
  EpiArgs e;
  e.Xt = bufs->x[st->ix];
  e.Y = bufs->x[st->io];
  e.LPY = bufs->lp[st->io];
  e.Y2 = st->dual ? bufs->x[st->io2] : nullptr;
  e.d2 = st->d2;
  e.d1 = st->d1;
  e.d0 = st->d0;
  e.lowp_kind = st->write_lowp ? (st->mode == SNF_P_BF16_REF64 ? kPrecBF16 : kPrecF32) : -1;
  e.want_e = st->want_e;
  e.c2 = st->c2;
  e.c1 = st->c1;
  e.c0 = st->c0;
  return e;
}

// Epilogue of one product entry p at global (r, c), x = X[r][c] (loaded by the caller, ahead
// of the stores, so that the loads of many entries are in flight together: the compiler may not
// move a load of X above a store to Y, which it cannot tell apart): Y = c2 p + c1 X +
// c0 [r == c], the FP64 sums, the mirror write.  In symmetric mode a diagonal tile keeps its
// upper half and mirrors it, so the result is exactly symmetric; every off-diagonal entry then
// stands for two.  With DUAL the second output Y2 is written too (compiled only into the
// kernel variants that need it, so the others keep their register budget).
template <bool DUAL = false>
__device__ __forceinline__ void epi_elem(double p, double x, int64_t r, int64_t c, int sym,
                                         int diag, int64_t n, int64_t np, const EpiArgs& ea,
                                         double& e2, double& t1, double& t2) {
  if (diag && sym && r > c) return;
  const bool mirror = sym && r != c;
  const double w = mirror ? 2.0 : 1.0;
  if (ea.want_e) {
    const double d = p - x;
    e2 += w * (d * d);
  }
  double y = ea.c2 * p + ea.c1 * x + (r == c ? ea.c0 : 0.0);
  if (r >= n || c >= n) y = 0.0;
  if (r == c) t1 += y;
  t2 += w * (y * y);
  ea.Y[r * np + c] = y;
  if (mirror) ea.Y[c * np + r] = y;
  if (DUAL && ea.Y2) {
    double y2 = ea.d2 * p + ea.d1 * x + (r == c ? ea.d0 : 0.0);
    if (r >= n || c >= n) y2 = 0.0;
    ea.Y2[r * np + c] = y2;
    if (mirror) ea.Y2[c * np + r] = y2;
  }
  if (ea.lowp_kind == kPrecF32) {
    const float yf = (float)y;
    ((float*)ea.LPY)[r * np + c] = yf;
    if (mirror) ((float*)ea.LPY)[c * np + r] = yf;
  } else if (ea.lowp_kind == kPrecBF16) {
    const unsigned short yb = f32_to_bf16_rne((float)y);
    ((unsigned short*)ea.LPY)[r * np + c] = yb;
    if (mirror) ((unsigned short*)ea.LPY)[c * np + r] = yb;
  }
}

// Row of accumulator register v of lane l inside its 16x16 MFMA block:
//   4 (l / 16) + v   for the f32 and bf16 MFMAs (ROWS_INTERLEAVED = false),
//   (l / 16) + 4 v   for the f64 MFMA          (ROWS_INTERLEAVED = true);
// the column is l % 16 for all three.
template <bool ROWS_INTERLEAVED>
__device__ __forceinline__ int acc_row(int lane, int v) {
  return ROWS_INTERLEAVED ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}

// Off-diagonal tile of a symmetric product in the f32 / bf16 accumulator layout: the lane's
// four values are rows r0 .. r0 + 3 of column c, so their mirror entries Y[c][r0 .. r0 + 3] are
// contiguous and go out as two 16-byte stores (and one 16- or 8-byte store of the
// low-precision copy) instead of four scattered 8-byte ones.  Same values as epi_elem.
template <typename Acc4>
__device__ __forceinline__ void epi_quad_mirrored(const Acc4& acc4, const double (&x4)[4],
                                                  int64_t r0, int64_t c, int64_t n, int64_t np,
                                                  const EpiArgs& ea, double& e2, double& t2) {
  double y[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t r = r0 + v;
    const double p = (double)acc4[v];
    const double x = x4[v];
    if (ea.want_e) {
      const double d = p - x;
      e2 += 2.0 * (d * d);
    }
    double yv = ea.c2 * p + ea.c1 * x;      // r != c in an off-diagonal tile
    if (r >= n || c >= n) yv = 0.0;
    t2 += 2.0 * (yv * yv);
    ea.Y[r * np + c] = yv;
    y[v] = yv;
  }
  double* ym = ea.Y + c * np + r0;
  *(double2*)(ym) = double2{y[0], y[1]};
  *(double2*)(ym + 2) = double2{y[2], y[3]};
  if (ea.lowp_kind == kPrecF32) {
    float* lp = (float*)ea.LPY;
    float f[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      f[v] = (float)y[v];
      lp[(r0 + v) * np + c] = f[v];
    }
    *(float4*)(lp + c * np + r0) = float4{f[0], f[1], f[2], f[3]};
  } else if (ea.lowp_kind == kPrecBF16) {
    unsigned short* lp = (unsigned short*)ea.LPY;
    unsigned short b[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      b[v] = f32_to_bf16_rne((float)y[v]);
      lp[(r0 + v) * np + c] = b[v];
    }
    *(uint2*)(lp + c * np + r0) = uint2{(unsigned)b[0] | ((unsigned)b[1] << 16),
                                        (unsigned)b[2] | ((unsigned)b[3] << 16)};
  }
}

// X[r][c] of the four entries of MFMA block (m, q) held by this lane.
template <bool ROWS_INTERLEAVED>
__device__ __forceinline__ void load_x_block(double (&x4)[4], int m, int q, int gi0, int gj0,
                                             int64_t np, const EpiArgs& ea) {
  const int lane = threadIdx.x & 63;
  const int64_t c = gj0 + q * 16 + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v)
    x4[v] = ea.Xt[(gi0 + m * 16 + acc_row<ROWS_INTERLEAVED>(lane, v)) * np + c];
}

// One 16x16 MFMA block (m, q) of the wave tile: acc4 holds its four values of this lane, x4
// the matching entries of X.
template <bool ROWS_INTERLEAVED, bool DUAL, typename Acc4>
__device__ __forceinline__ void epilogue_block(const Acc4& acc4, const double (&x4)[4], int m,
                                               int q, int gi0, int gj0, int sym, int diag,
                                               int64_t n, int64_t np, const EpiArgs& ea,
                                               double& e2, double& t1, double& t2) {
  const int lane = threadIdx.x & 63;
  const int64_t c = gj0 + q * 16 + (lane & 15);
  if (!ROWS_INTERLEAVED && !DUAL && sym && !diag) {
    epi_quad_mirrored(acc4, x4, gi0 + m * 16 + acc_row<false>(lane, 0), c, n, np, ea, e2, t2);
    return;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t r = gi0 + m * 16 + acc_row<ROWS_INTERLEAVED>(lane, v);
    epi_elem<DUAL>((double)acc4[v], x4[v], r, c, sym, diag, n, np, ea, e2, t1, t2);
  }
}

// The wave tile's epilogue.  X values are loaded in batches ahead of the stores: BATCH -1
// loads each value just before its entry's stores, 0 the four values of one MFMA block before
// that block's stores, 1 those of a row of blocks before the row's stores, 2 also the next
// row's before the current row's stores (more registers each: the FP64 kernels, at 4 waves per
// SIMD, have room only for -1).
template <bool ROWS_INTERLEAVED, bool DUAL, int BATCH = 0, int MT, int QT, typename AccT>
__device__ __forceinline__ void epilogue(const AccT (&acc)[MT][QT], int gi0, int gj0, int sym,
                                         int diag, int64_t n, int64_t np, const EpiArgs& ea,
                                         double& e2, double& t1, double& t2) {
  if constexpr (BATCH < 0) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        const int64_t c = gj0 + q * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = gi0 + m * 16 + acc_row<ROWS_INTERLEAVED>(lane, v);
          if (diag && sym && r > c) continue;   // (the entry's mirror is written instead)
          epi_elem<DUAL>((double)acc[m][q][v], ea.Xt[r * np + c], r, c, sym, diag, n, np, ea,
                         e2, t1, t2);
        }
      }
  } else if constexpr (BATCH == 0) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        double x4[4];
        load_x_block<ROWS_INTERLEAVED>(x4, m, q, gi0, gj0, np, ea);
        epilogue_block<ROWS_INTERLEAVED, DUAL>(acc[m][q], x4, m, q, gi0, gj0, sym, diag, n, np,
                                               ea, e2, t1, t2);
      }
  } else {
    constexpr int NB = BATCH == 2 ? 2 : 1;
    double xs[NB][QT][4];
    if (BATCH == 2) {
#pragma unroll
      for (int q = 0; q < QT; ++q)
        load_x_block<ROWS_INTERLEAVED>(xs[0][q], 0, q, gi0, gj0, np, ea);
    }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int nm = BATCH == 2 ? m + 1 : m;
      if (nm < MT) {
#pragma unroll
        for (int q = 0; q < QT; ++q)
          load_x_block<ROWS_INTERLEAVED>(xs[nm % NB][q], nm, q, gi0, gj0, np, ea);
      }
#pragma unroll
      for (int q = 0; q < QT; ++q)
        epilogue_block<ROWS_INTERLEAVED, DUAL>(acc[m][q], xs[m % NB][q], m, q, gi0, gj0, sym,
                                               diag, n, np, ea, e2, t1, t2);
    }
  }
}

__device__ __forceinline__ void write_partials(double e2, double t1, double t2,
                                               double* partials, int tile) {
  __shared__ double red[24];
  block_sum3(e2, t1, t2, red);
  if (threadIdx.x == 0) {
    partials[tile * 4 + 0] = e2;
    partials[tile * 4 + 1] = t1;
    partials[tile * 4 + 2] = t2;
    partials[tile * 4 + 3] = 0.0;
  }
}

// Work decomposition of one product launch.  Workgroups [0, dp_tiles) compute whole tiles
// (id remapped per XCD); the remaining workgroups compute one of split_s k-slices of the
// tail tiles [dp_tiles, dp_tiles + tail_tiles) and store their raw accumulators; the
// fix-up kernel adds the slices of a tile in a fixed order and runs the epilogue.
struct WorkItem {
  int tile;
  int piece;     // -1 for a whole tile, else the slice's index into the split buffer
  int kt_begin, kt_end;
};

__device__ __forceinline__ WorkItem work_item(const ProductGrid& g, int KT) {
  WorkItem it;
  const int w = blockIdx.x;
  if (w < g.dp_tiles) {
    it.tile = xcd_remap(w, g.dp_tiles);
    it.piece = -1;
    it.kt_begin = 0;
    it.kt_end = KT;
  } else {
    const int q = w - g.dp_tiles;
    const int p = q % g.split_s;
    it.tile = g.dp_tiles + q / g.split_s;
    it.piece = q;
    it.kt_begin = (int)((int64_t)p * KT / g.split_s);
    it.kt_end = (int)((int64_t)(p + 1) * KT / g.split_s);
  }
  return it;
}

// Raw accumulators of a k-slice in tile order: split[piece][r][c], r, c < 128, whatever the
// thread layout of the kernel that produced them.
template <bool ROWS_INTERLEAVED, int MT, int QT, typename AccT>
__device__ __forceinline__ void store_slice(const AccT (&acc)[MT][QT], int wr0, int wc0,
                                            double* split, int piece) {
  const int lane = threadIdx.x & 63;
  double* base = split + (size_t)piece * kTile * kTile;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int q = 0; q < QT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr0 + m * 16 + acc_row<ROWS_INTERLEAVED>(lane, v);
        const int c = wc0 + q * 16 + (lane & 15);
        base[r * kTile + c] = (double)acc[m][q][v];
      }
}

// ---------------------------------------------------------------------------------------
// Product kernel, f64 / f32 MFMA 16x16x4.
//   LDS tiles hold 'k-rows' of both operands: sA[k][i] = A[k0+k][i0+i] and
//   sB[k][j] = B[k0+k][j0+j]; A[i][k] = A[k][i] because A is symmetric, so both panels are
//   read with contiguous, coalesced rows.  MFMA operand of lane l: row/col (l % 16), k (l / 16).
// ---------------------------------------------------------------------------------------
// Thread layout: NT threads = (NT/64) waves in WR x WC, each wave a (128/WR) x (128/WC)
// piece of the tile made of MT x QT MFMA 16x16 blocks.
template <typename T> struct Layout;
template <> struct Layout<double> {   // 8 waves of 64x32: 64 accumulator registers per lane,
  static constexpr int NT = 512, WC = 4;   // so 4 waves fit on each SIMD
};
template <> struct Layout<float> {    // 8 waves of 32x64: 32 accumulator registers per lane,
  static constexpr int NT = 512, WC = 2;   // 4 waves per SIMD
};

template <typename T, int PREC, bool DUAL = false>
__device__ __forceinline__ void product_body(const SnfState* __restrict__ st,
                                             const Buffers* __restrict__ bufs,
                                             const ProductGrid& g, const WorkItem& wi) {
  typedef Mfma<T> M;
  constexpr int NT = Layout<T>::NT, WC = Layout<T>::WC, WR = NT / 64 / WC;
  constexpr int TR = kTile / WR, TC = kTile / WC, MT = TR / 16, QT = TC / 16;
  constexpr int BK = M::kBK, LDS_W = kTile + M::kPad;
  constexpr int VE = 16 / sizeof(T);          // elements per 16-byte vector
  constexpr int VPR = kTile / VE;             // vectors per LDS row
  constexpr int RPP = NT / VPR;               // rows per load pass
  constexpr int PASSES = BK / RPP;
  __shared__ __attribute__((aligned(16))) T sA[2][BK][LDS_W];
  __shared__ __attribute__((aligned(16))) T sB[2][BK][LDS_W];

  const int64_t np = g.np;
  const T* A = (PREC == kPrecF64) ? (const T*)bufs->x[st->ia] : (const T*)bufs->lp[st->ia];
  const T* B = (PREC == kPrecF64) ? (const T*)bufs->x[st->ib] : (const T*)bufs->lp[st->ib];

  int bi, bj;
  tile_coords(wi.tile, (int)(np / kTile), g.sym, bi, bj);
  const int64_t i0 = (int64_t)bi * kTile, j0 = (int64_t)bj * kTile;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid / WC, wc = wid % WC;
  const int lrow = tid / VPR, lvec = tid % VPR;

  typename M::acc_t acc[MT][QT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int q = 0; q < QT; ++q) acc[m][q] = typename M::acc_t{0, 0, 0, 0};

  u32x4 ra0[PASSES], rb0[PASSES], ra1[PASSES], rb1[PASSES];
  auto gload = [&](u32x4 (&ra)[PASSES], u32x4 (&rb)[PASSES], int64_t k0) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const int64_t k = k0 + p * RPP + lrow;
      ra[p] = gload16(A + k * np + i0 + lvec * VE);
      rb[p] = gload16(B + k * np + j0 + lvec * VE);
    }
  };
  auto lstore = [&](const u32x4 (&ra)[PASSES], const u32x4 (&rb)[PASSES], int buf) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      *(u32x4*)(&sA[buf][p * RPP + lrow][lvec * VE]) = ra[p];
      *(u32x4*)(&sB[buf][p * RPP + lrow][lvec * VE]) = rb[p];
    }
  };
  const int fr = lane & 15, fk = lane >> 4;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[MT], b[QT];
#pragma unroll
      for (int m = 0; m < MT; ++m) a[m] = sA[buf][kk + fk][wr * TR + m * 16 + fr];
#pragma unroll
      for (int q = 0; q < QT; ++q) b[q] = sB[buf][kk + fk][wc * TC + q * 16 + fr];
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int q = 0; q < QT; ++q) acc[m][q] = M::mma(a[m], b[q], acc[m][q]);
    }
  };
  // FP32: operands two stages ahead in two register sets, the loads issued on every path
  // (past the end the last stage again, never stored) so that the wait before the LDS stores
  // leaves the newer set in flight.  FP64: one stage ahead (a stage's 32 MFMAs per wave take
  // long enough to cover the loads, and the FP64 kernel has no registers to spare).
  const int kb = wi.kt_begin, ke = wi.kt_end;
  gload(ra0, rb0, (int64_t)kb * BK);
  lstore(ra0, rb0, 0);
  if constexpr (PREC == kPrecF32) {
    gload(ra1, rb1, (int64_t)min(kb + 1, ke - 1) * BK);
    __syncthreads();
    int kt = kb;
    while (true) {
      {
        const int buf = (kt - kb) & 1;
        gload(ra0, rb0, (int64_t)min(kt + 2, ke - 1) * BK);
        compute(buf);
        if (kt + 1 < ke) lstore(ra1, rb1, buf ^ 1);
        __syncthreads();
        if (++kt >= ke) break;
      }
      {
        const int buf = (kt - kb) & 1;
        gload(ra1, rb1, (int64_t)min(kt + 2, ke - 1) * BK);
        compute(buf);
        if (kt + 1 < ke) lstore(ra0, rb0, buf ^ 1);
        __syncthreads();
        if (++kt >= ke) break;
      }
    }
  } else {
    __syncthreads();
    for (int kt = kb; kt < ke; ++kt) {
      const int buf = (kt - kb) & 1;
      const bool more = kt + 1 < ke;
      if (more) gload(ra0, rb0, (int64_t)(kt + 1) * BK);
      compute(buf);
      if (more) lstore(ra0, rb0, buf ^ 1);
      __syncthreads();
    }
  }

  if (wi.piece >= 0) {
    store_slice<PREC == kPrecF64>(acc, wr * TR, wc * TC, g.split_buf, wi.piece);
    return;
  }
  const EpiArgs ea = epi_args(st, bufs);
  double e2 = 0.0, t1 = 0.0, t2 = 0.0;
  epilogue<PREC == kPrecF64, DUAL, PREC == kPrecF64 ? -1 : 0>(acc, (int)(i0 + wr * TR),
                                                             (int)(j0 + wc * TC), g.sym,
                                   bi == bj, g.n, np, ea, e2, t1, t2);
  write_partials(e2, t1, t2, g.partials, wi.tile);
}

// ---------------------------------------------------------------------------------------
// Small orders: FP64 product in 32x32 output tiles with the k range split over the four
// waves of a workgroup and summed in LDS, so a step needs no split fix-up launch (at
// n = 256 the 128x128 engine has 3 tiles, which it splits 16 ways and then fixes up).
// Wave w sums k in [w np/4, (w + 1) np/4) in chunks of 32; in MFMA step s of a chunk the lane
// group g = l / 16 takes k = chunk + 8 g + s, so each lane reads 8 consecutive values of a
// row (operands are symmetric: row j of B is column j).  The four partial tiles are added
// in wave order, then the shared epilogue runs on 4 entries per thread.
// ---------------------------------------------------------------------------------------
constexpr int kSmallTile = 32;
constexpr int kSmallThreads = 256;

// One 32x32 tile of the pending product (st: the scalar state, in device memory or an LDS
// copy of it); its FP64 sums go to partials[tile].
__device__ __forceinline__ void small_tile_product(const SnfState* __restrict__ st,
                                                   const Buffers* __restrict__ bufs,
                                                   const SmallGrid& g, int tile,
                                                   double* __restrict__ partials,
                                                   double (*part)[kSmallTile][kSmallTile + 1]) {
  const int64_t np = g.np;
  const double* A = bufs->x[st->ia];
  const double* B = bufs->x[st->ib];
  int bi, bj;
  tile_coords(tile, (int)(np / kSmallTile), 1, bi, bj);
  const int64_t i0 = (int64_t)bi * kSmallTile, j0 = (int64_t)bj * kSmallTile;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int fr = lane & 15, fg = lane >> 4;
  const int64_t kw0 = (int64_t)wid * (np / 4), kw1 = kw0 + np / 4;

  dbl4 acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[m][q] = dbl4{0.0, 0.0, 0.0, 0.0};

  // chunk registers: rows m (A) and q (B), 8 consecutive k values each (4 x 16 bytes); two
  // sets, so the next chunk's loads are in flight while this one's MFMAs run
  u32x4 ra0[2][4], rb0[2][4], ra1[2][4], rb1[2][4];
  auto gload = [&](int64_t kc, u32x4 (&ra)[2][4], u32x4 (&rb)[2][4]) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const double* pa = A + (i0 + m * 16 + fr) * np + kc + fg * 8;
      const double* pb = B + (j0 + m * 16 + fr) * np + kc + fg * 8;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ra[m][v] = gload16(pa + 2 * v);
        rb[m][v] = gload16(pb + 2 * v);
      }
    }
  };
  auto compute = [&](const u32x4 (&ra)[2][4], const u32x4 (&rb)[2][4]) {
    double a[2][8], b[2][8];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double2 da = __builtin_bit_cast(double2, ra[m][v]);
        const double2 db = __builtin_bit_cast(double2, rb[m][v]);
        a[m][2 * v] = da.x;
        a[m][2 * v + 1] = da.y;
        b[m][2 * v] = db.x;
        b[m][2 * v + 1] = db.y;
      }
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m][s], b[q][s], acc[m][q], 0, 0, 0);
  };
  // the wave's range is a multiple of 32 (np is a multiple of 128).  The next chunk is
  // loaded on every path (past the end the last chunk again, never used) and ahead of this
  // chunk's MFMAs (scheduling barrier): with a conditional load the compiler's wait before
  // the MFMAs would also cover the next chunk's loads, and they would not overlap.
  gload(kw0, ra0, rb0);
  for (int64_t kc = kw0; kc < kw1; kc += 64) {
    gload(min(kc + 32, kw1 - 32), ra1, rb1);
    __builtin_amdgcn_sched_barrier(0);
    compute(ra0, rb0);
    gload(min(kc + 64, kw1 - 32), ra0, rb0);
    __builtin_amdgcn_sched_barrier(0);
    if (kc + 32 < kw1) compute(ra1, rb1);
  }
  // accumulator of lane l, register v: row (l / 16) + 4 v, column l % 16 of block (m, q)
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        part[wid][m * 16 + fg + 4 * v][q * 16 + fr] = acc[m][q][v];
  __syncthreads();
  const EpiArgs ea = epi_args(st, bufs);
  double e2 = 0.0, t1 = 0.0, t2 = 0.0;
  double xs[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int idx = e * kSmallThreads + tid;
    xs[e] = ea.Xt[(i0 + idx / kSmallTile) * np + j0 + idx % kSmallTile];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int idx = e * kSmallThreads + tid;
    const int r = idx / kSmallTile, c = idx % kSmallTile;
    const double p = ((part[0][r][c] + part[1][r][c]) + part[2][r][c]) + part[3][r][c];
    epi_elem(p, xs[e], i0 + r, j0 + c, 1, bi == bj, g.n, np, ea, e2, t1, t2);
  }
  write_partials(e2, t1, t2, partials, tile);
}

__global__ __launch_bounds__(kSmallThreads) void product_f64_small_kernel(
    const SnfState* __restrict__ st, const Buffers* __restrict__ bufs, SmallGrid g) {
  if (st->stop || st->prec != kPrecF64 || st->dual) return;
  __shared__ double part[4][kSmallTile][kSmallTile + 1];
  small_tile_product(st, bufs, g, blockIdx.x, g.partials, part);
}


SmallGrid make_small_grid(int64_t np, int64_t n, double* partials) {
  SmallGrid g;
  g.np = np;
  g.n = n;
  g.partials = partials;
  const int nt = (int)(np / kSmallTile);
  g.tiles = nt * (nt + 1) / 2;
  return g;
}

void launch_product_small(SnfState* st, const Buffers* bufs_dev, const SmallGrid& g,
                          hipStream_t s) {
  hipLaunchKernelGGL(product_f64_small_kernel, dim3(g.tiles), dim3(kSmallThreads), 0, s, st,
                     bufs_dev, g);
}

// ---------------------------------------------------------------------------------------
// Product kernel, bf16 MFMA 16x16x32 with f32 accumulation.
//   Here the LDS tiles are 'row panels' with k contiguous: sA[i][k] = A[i0+i][k0+k] and
//   sB[j][k] = B[j0+j][k0+k] (B[k][j] = B[j][k] by symmetry), because a lane's MFMA operand
//   is 8 consecutive k values of one row / column: lane l holds row (l % 16),
//   k = 8 (l / 16) .. 8 (l / 16) + 7.  Rows are 128 bytes (eight 16-byte chunks) without
//   padding; chunk c of row r is stored at position c ^ ((r >> 1) & 7), so that both the
//   stores (two rows of eight chunks per 16 lanes) and the operand reads (16 rows, one chunk
//   each) hit every bank once.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void product_bf16_body(const SnfState* __restrict__ st,
                                                  const Buffers* __restrict__ bufs,
                                                  const ProductGrid& g, const WorkItem& wi) {
  constexpr int BK = 64;                 // bf16 per LDS row per stage = 128 B
  constexpr int LDS_W = BK;              // row stride 128 B, chunks swizzled
  constexpr int VPR = BK / 8;            // 16-byte vectors per row = 8
  constexpr int RPP = kThreads / VPR;    // 32 rows per pass
  constexpr int PASSES = kTile / RPP;    // 4
  __shared__ __attribute__((aligned(16))) unsigned short sA[2][kTile][LDS_W];
  __shared__ __attribute__((aligned(16))) unsigned short sB[2][kTile][LDS_W];

  const int64_t np = g.np;
  const unsigned short* A = (const unsigned short*)bufs->lp[st->ia];
  const unsigned short* B = (const unsigned short*)bufs->lp[st->ib];

  int bi, bj;
  tile_coords(wi.tile, (int)(np / kTile), g.sym, bi, bj);
  const int64_t i0 = (int64_t)bi * kTile, j0 = (int64_t)bj * kTile;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int lrow = tid / VPR, lvec = tid % VPR;

  flt4 acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[m][q] = flt4{0.f, 0.f, 0.f, 0.f};

  u32x4 ra0[PASSES], rb0[PASSES], ra1[PASSES], rb1[PASSES];
  auto gload = [&](u32x4 (&ra)[PASSES], u32x4 (&rb)[PASSES], int64_t k0) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const int64_t r = p * RPP + lrow;
      ra[p] = gload16(A + (i0 + r) * np + k0 + lvec * 8);
      rb[p] = gload16(B + (j0 + r) * np + k0 + lvec * 8);
    }
  };
  auto lstore = [&](const u32x4 (&ra)[PASSES], const u32x4 (&rb)[PASSES], int buf) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const int rr = p * RPP + lrow, pc = (lvec ^ ((rr >> 1) & 7)) * 8;
      *(u32x4*)(&sA[buf][rr][pc]) = ra[p];
      *(u32x4*)(&sB[buf][rr][pc]) = rb[p];
    }
  };
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      bf16x8 a[4], b[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int rr = wr * 64 + m * 16 + fr;
        a[m] = *(const bf16x8*)(&sA[buf][rr][(((kk + fk) >> 3) ^ ((rr >> 1) & 7)) * 8]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = wc * 64 + q * 16 + fr;
        b[q] = *(const bf16x8*)(&sB[buf][rr][(((kk + fk) >> 3) ^ ((rr >> 1) & 7)) * 8]);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc[m][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b[q], acc[m][q], 0, 0, 0);
    }
  };

  // Operands two stages ahead in two register sets: stage kt computes from LDS buffer
  // (kt - kb) & 1, stores stage kt + 1 (loaded during the previous stage) into the other
  // buffer and loads stage kt + 2.  The loads are issued on every path (past the end the
  // last stage again, never stored): with a conditional load the compiler's wait before the
  // LDS stores would also cover the newer set and the second stage of lead would be lost.
  const int kb = wi.kt_begin, ke = wi.kt_end;
  gload(ra0, rb0, (int64_t)kb * BK);
  lstore(ra0, rb0, 0);
  gload(ra1, rb1, (int64_t)min(kb + 1, ke - 1) * BK);
  __syncthreads();
  int kt = kb;
  while (true) {
    {
      const int buf = (kt - kb) & 1;
      gload(ra0, rb0, (int64_t)min(kt + 2, ke - 1) * BK);
      compute(buf);
      if (kt + 1 < ke) lstore(ra1, rb1, buf ^ 1);
      __syncthreads();
      if (++kt >= ke) break;
    }
    {
      const int buf = (kt - kb) & 1;
      gload(ra1, rb1, (int64_t)min(kt + 2, ke - 1) * BK);
      compute(buf);
      if (kt + 1 < ke) lstore(ra0, rb0, buf ^ 1);
      __syncthreads();
      if (++kt >= ke) break;
    }
  }

  if (wi.piece >= 0) {
    store_slice<false>(acc, wr * 64, wc * 64, g.split_buf, wi.piece);
    return;
  }
  const EpiArgs ea = epi_args(st, bufs);
  double e2 = 0.0, t1 = 0.0, t2 = 0.0;
  epilogue<false, false, 2>(acc, (int)(i0 + wr * 64), (int)(j0 + wc * 64), g.sym, bi == bj,
                            g.n,
                         np, ea, e2, t1, t2);
  write_partials(e2, t1, t2, g.partials, wi.tile);
}

__global__ __launch_bounds__(512, 2) void product_f64_kernel(const SnfState* __restrict__ st,
                                                             const Buffers* __restrict__ bufs,
                                                             ProductGrid g) {
  if (st->stop || st->prec != kPrecF64 || st->dual) return;
  product_body<double, kPrecF64>(st, bufs, g, work_item(g, (int)(g.np / Mfma<double>::kBK)));
}

// The FP64 product whose epilogue also writes the second output (the first product of a
// P_{i,j} iteration); the host launches it beside product_f64_kernel for those schemes and
// exactly one of the two runs.
__global__ __launch_bounds__(512, 2) void product_f64_dual_kernel(const SnfState* __restrict__ st,
                                                                  const Buffers* __restrict__ bufs,
                                                                  ProductGrid g) {
  if (st->stop || st->prec != kPrecF64 || !st->dual) return;
  product_body<double, kPrecF64, true>(st, bufs, g,
                                       work_item(g, (int)(g.np / Mfma<double>::kBK)));
}

__global__ __launch_bounds__(512, 2) void product_f32_kernel(const SnfState* __restrict__ st,
                                                             const Buffers* __restrict__ bufs,
                                                             ProductGrid g) {
  if (st->stop || st->prec != kPrecF32) return;
  product_body<float, kPrecF32>(st, bufs, g, work_item(g, (int)(g.np / Mfma<float>::kBK)));
}

__global__ __launch_bounds__(256, 2) void product_bf16_kernel(const SnfState* __restrict__ st,
                                                              const Buffers* __restrict__ bufs,
                                                              ProductGrid g) {
  if (st->stop || st->prec != kPrecBF16) return;
  product_bf16_body(st, bufs, g, work_item(g, (int)(g.np / 64)));
}

// Fix-up of the split tail tiles: workgroup (t, b) handles rows 8b .. 8b + 7 of tail tile t
// (256 threads, 4 consecutive columns each); it adds the k-slices in slice order (the loads
// of four slices in flight at a time), runs the epilogue of those entries and stores its
// sums in its own partials slot.
constexpr int kMaxSplit = 16;
__global__ __launch_bounds__(256) void split_fixup_kernel(const SnfState* __restrict__ st,
                                                          const Buffers* __restrict__ bufs,
                                                          ProductGrid g) {
  if (st->stop) return;
  const int t = blockIdx.x >> 4, b = blockIdx.x & 15;
  const int tile = g.dp_tiles + t;
  int bi, bj;
  tile_coords(tile, (int)(g.np / kTile), g.sym, bi, bj);
  const int r = 8 * b + (threadIdx.x >> 5), c0 = (threadIdx.x & 31) * 4;
  const double* base = g.split_buf + (size_t)t * g.split_s * kTile * kTile + r * kTile + c0;
  double sum[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p0 = 0; p0 < g.split_s; p0 += 4) {
    double part[4][4];
#pragma unroll
    for (int pp = 0; pp < 4; ++pp)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        part[pp][v] = (p0 + pp < g.split_s) ? base[(size_t)(p0 + pp) * kTile * kTile + v] : 0.0;
#pragma unroll
    for (int pp = 0; pp < 4; ++pp)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (p0 + pp < g.split_s) sum[v] += part[pp][v];
  }
  const EpiArgs ea = epi_args(st, bufs);
  double e2 = 0.0, t1 = 0.0, t2 = 0.0;
  const int64_t gr = (int64_t)bi * kTile + r;
  double xs[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) xs[v] = ea.Xt[gr * g.np + (int64_t)bj * kTile + c0 + v];
#pragma unroll
  for (int v = 0; v < 4; ++v)
    epi_elem<true>(sum[v], xs[v], gr, (int64_t)bj * kTile + c0 + v, g.sym, bi == bj, g.n, g.np,
                   ea, e2, t1, t2);
  write_partials(e2, t1, t2, g.partials, g.dp_tiles + blockIdx.x);
}

ProductGrid make_product_grid(int64_t np, int64_t n, int sym, int num_cus, double* partials,
                              double* split_buf, int split_cap, int stage_depth) {
  ProductGrid g;
  g.np = np;
  g.n = n;
  g.sym = sym;
  g.partials = partials;
  g.split_buf = split_buf;
  const int tiles = num_product_tiles(np, sym);
  g.dp_tiles = tiles;
  g.tail_tiles = 0;
  g.split_s = 1;
  g.partial_count = tiles;
  if (num_cus <= 0 || !split_buf) return g;
  const int rem = tiles % num_cus;
  // every slice needs at least one k-stage of the deepest stage that may run (f64 16,
  // f32 32, bf16 64 values of k per stage)
  const int kt_min = (int)(np / stage_depth);
  if (rem == 0) return g;
  int s;
  if (rem <= num_cus / 2) {
    s = num_cus / rem;            // a short tail: one slice per compute unit
  } else if (tiles == rem) {
    // a single wave of more than half as many tiles as compute units: whole tiles would
    // run one workgroup per compute unit; three or more slices per tile fill both
    // workgroup slots of every unit (n = 2048: 136 tiles, 3 slices each).  A lone workgroup
    // already gets about half the unit's rate, so two slices per tile gain nothing.
    s = 2 * num_cus / rem;
    if (s < 3) return g;
  } else {
    return g;                     // a long tail behind full waves: whole tiles
  }
  if (s > kt_min) s = kt_min;
  if (s > kMaxSplit) s = kMaxSplit;
  if (s < 2 || rem * s > split_cap) return g;
  g.dp_tiles = tiles - rem;
  g.tail_tiles = rem;
  g.split_s = s;
  g.partial_count = g.dp_tiles + 16 * rem;   // one slot per fix-up workgroup
  return g;
}

void launch_product(int prec, SnfState* st, const Buffers* bufs_dev, const ProductGrid& g,
                    hipStream_t s) {
  const int grid = g.dp_tiles + g.tail_tiles * g.split_s;
  if (prec == kPrecF64) {
    hipLaunchKernelGGL(product_f64_kernel, dim3(grid), dim3(Layout<double>::NT), 0, s, st,
                       bufs_dev, g);
  } else if (prec == kPrecF32) {
    hipLaunchKernelGGL(product_f32_kernel, dim3(grid), dim3(Layout<float>::NT), 0, s, st,
                       bufs_dev, g);
  } else {
    hipLaunchKernelGGL(product_bf16_kernel, dim3(grid), dim3(kThreads), 0, s, st, bufs_dev, g);
  }
}

void launch_product_dual(SnfState* st, const Buffers* bufs_dev, const ProductGrid& g,
                         hipStream_t s) {
  const int grid = g.dp_tiles + g.tail_tiles * g.split_s;
  hipLaunchKernelGGL(product_f64_dual_kernel, dim3(grid), dim3(Layout<double>::NT), 0, s, st,
                     bufs_dev, g);
}

void launch_split_fixup(SnfState* st, const Buffers* bufs_dev, const ProductGrid& g,
                        hipStream_t s) {
  if (g.tail_tiles == 0) return;
  hipLaunchKernelGGL(split_fixup_kernel, dim3(g.tail_tiles * 16), dim3(kThreads), 0, s, st,
                     bufs_dev, g);
}
// ---------------------------------------------------------------------------------------
// Schedule: reduce the partials in a fixed order, then advance the scalar state.
// ---------------------------------------------------------------------------------------
// alpha of a scaled P_{i,j} step: the smaller of the two sides' roots (tables from the state)
__device__ double pij_alpha_state(const SnfState* s) {
  const double lo = sched::pij_alpha_side_tab(s->pij_i, s->pij_j, s->pbin[0], s->xstar, s->beta);
  const double hi =
      sched::pij_alpha_side_tab(s->pij_j, s->pij_i, s->pbin[1], 1.0 - s->xstar, s->abar);
  return lo < hi ? lo : hi;
}

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
  s->dual = 0;
  if (scheme_is_pij(scheme)) {
    br = SNF_BRANCH_PIJ;
    a = (scheme == SNF_SNF_FIXMU_PIJ)
            ? pij_alpha_state(s)
            : 1.0;
  } else if (scheme == SNF_SP2_TRACE) {
    br = sched::trace_square(s->t1, s->t2, (double)s->n_occ) ? SNF_BRANCH_SQUARE
                                                             : SNF_BRANCH_FOLD;
  } else if (scheme == SNF_TC2_BETA || scheme == SNF_SNF_VARMU) {
    const bool sq = sched::alg2_square(s->beta, s->betabar);
    br = sq ? SNF_BRANCH_SQUARE : SNF_BRANCH_FOLD;
    if (scheme == SNF_SNF_VARMU)
      a = sq ? sched::alg2_square_alpha(s->beta) : sched::alg2_fold_alpha(s->betabar);
  } else if (scheme_pmm_m(scheme)) {
    br = s->pmm_m == 3 ? SNF_BRANCH_P33 : SNF_BRANCH_P55;
    a = (scheme == SNF_SNF_FIXMU3 || scheme == SNF_SNF_FIXMU5)
            ? sched::pmm_alpha_tab(s->pmm_m, s->pbin[0], s->beta)
                                                               : 1.0;
  } else {
    br = SNF_BRANCH_P11;
    a = (scheme == SNF_SNF_FIXMU) ? sched::alg1_alpha(s->beta) : 1.0;
  }
  s->branch = br;
  s->alpha = a;
  if (br == SNF_BRANCH_PIJ) {
    // W = V^2, V = a (X - x* I): W = a^2 P - 2 a^2 x* X + a^2 x*^2 I; and beside it the top
    // Horner level T = q_2h W + q_(2h-1) V + q_(2h-2) I in the same epilogue
    const double xs = s->xstar, a2 = a * a;
    const int h = (s->pij_i + s->pij_j) / 2;
    const double qt = s->pq[2 * h], qo = s->pq[2 * h - 1], qc = s->pq[2 * h - 2];
    s->c2 = a2;
    s->c1 = -2.0 * a2 * xs;
    s->c0 = a2 * xs * xs;
    s->d2 = qt * a2;
    s->d1 = qo * a - 2.0 * qt * a2 * xs;
    s->d0 = qt * a2 * xs * xs - qo * a * xs + qc;
  } else if (br == SNF_BRANCH_P33 || br == SNF_BRANCH_P55) {
    // W = (a (X - I/2))^2 = a^2 P - a^2 X + (a^2 / 4) I
    const double a2 = a * a;
    s->c2 = a2;
    s->c1 = -a2;
    s->c0 = 0.25 * a2;
  } else if (br == SNF_BRANCH_SQUARE) {          // ((1+a) X - a I)^2 = (1+a)^2 P - 2a(1+a) X + a^2 I
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
  if (br == SNF_BRANCH_P33 || br == SNF_BRANCH_P55) {
    s->bw = (s->cur + 1) & 3;
    s->io = s->bw;
    s->horner_left = s->pmm_m - 1;
  } else if (br == SNF_BRANCH_PIJ) {
    s->bw = (s->cur + 1) & 3;
    s->io = s->bw;
    s->dual = 1;
    s->io2 = s->bt = (s->cur + 2) & 3;
    s->horner_left = (s->pij_i + s->pij_j) / 2 - 1;
  } else {
    s->io = (br == SNF_BRANCH_P11) ? 2 : 1 - s->cur;
  }
}

__device__ void advance_beta(SnfState* s, int br, double a) {
#pragma clang fp contract(off)
  if (br == SNF_BRANCH_SQUARE) {
    s->beta = sched::alg2_square_map(s->beta, a);
    s->betabar = sched::alg2_square_map(s->betabar, a);
  } else if (br == SNF_BRANCH_FOLD) {
    s->beta = sched::alg2_fold_map(s->beta, a);
    s->betabar = sched::alg2_fold_map(s->betabar, a);
  } else if (br == SNF_BRANCH_P11) {
    s->beta = sched::alg1_beta_next(s->beta, a);
    s->betabar = 1.0 - s->beta;
  } else if (br == SNF_BRANCH_PIJ) {
    const double xs = s->xstar;
    const double an = sched::pij_side_next_tab(s->pij_i, s->pij_j, s->pbin[0], xs, s->beta, a);
    const double bn =
        sched::pij_side_next_tab(s->pij_j, s->pij_i, s->pbin[1], 1.0 - xs, s->abar, a);
    s->beta = an;
    s->abar = bn;
    s->betabar = 1.0 - bn;
  } else {
    s->beta = sched::pij_eval_tab(s->pmm_m, s->pmm_m, s->pbin[0], a * (s->beta - 0.5) + 0.5);
    s->betabar = 1.0 - s->beta;
  }
}

// Set up the next product of a P_{m,m} iteration once the previous one finished:
// P(1/2 + v) = 1/2 + v r(v^2), v = a (X - I/2), W = v^2.  After W: T = r_m W^2 + r_{m-1} W
// + r_{m-2} I from W.W; then T <- W.T + r_k I down to k = 0; then X_new = 1/2 I + v T.
__device__ void pmm_next(SnfState* s) {
#pragma clang fp contract(off)
  const int m = s->pmm_m;
  double r[sched::kPmmMaxM + 1];
  for (int k = 0; k <= m; ++k) r[k] = s->pr[k];
  const int ta = (s->cur + 2) & 3, tb = (s->cur + 3) & 3;
  s->want_e = 0;
  if (s->kind == kKindSquare) {             // W done: first Horner level from W.W
    s->kind = kKindHorner;
    s->ia = s->ib = s->ix = s->bw;
    s->io = s->bt = ta;
    s->c2 = r[m];
    s->c1 = r[m - 1];
    s->c0 = r[m - 2];
    return;
  }
  if (s->kind == kKindHorner && s->horner_left > 0) {   // T <- W.T + r_k I
    const int k = s->horner_left - 1;
    s->ia = s->bw;
    s->ib = s->ix = s->bt;
    s->io = (s->bt == ta) ? tb : ta;
    s->bt = s->io;
    s->c2 = 1.0;
    s->c1 = 0.0;
    s->c0 = r[k];
    return;
  }
  // T = r(W) done: X_new = a X.T - (a / 2) T + I / 2, written over W
  s->kind = kKindFinal;
  s->ia = s->cur;
  s->ib = s->ix = s->bt;
  s->io = s->bw;
  s->c2 = s->alpha;
  s->c1 = -0.5 * s->alpha;
  s->c0 = 0.5;
}

// Set up the next product of a P_{i,j} iteration: P(x* + v) = x* + v Q(v), v = a (X - x* I),
// W = v^2, Q(v) = sum_k (q_2k + q_(2k+1) v) W^k.  The first product gave W and the top level
// T; then T <- T.W + q_(2k+1) V + q_2k I for k = h - 2 .. 0; then X_new = x* I + V T.
__device__ void pij_next(SnfState* s) {
#pragma clang fp contract(off)
  const double a = s->alpha, xs = s->xstar;
  const int ta = (s->cur + 2) & 3, tb = (s->cur + 3) & 3;
  s->want_e = 0;
  s->dual = 0;
  if (s->horner_left > 0) {
    const int k = s->horner_left - 1;
    s->kind = kKindHorner;
    s->ia = s->bt;
    s->ib = s->bw;
    s->ix = s->cur;
    s->io = (s->bt == ta) ? tb : ta;
    s->bt = s->io;
    s->c2 = 1.0;
    s->c1 = s->pq[2 * k + 1] * a;
    s->c0 = s->pq[2 * k] - s->pq[2 * k + 1] * a * xs;
    return;
  }
  // X_new = a X.T - a x* T + x* I, written over W
  s->kind = kKindFinal;
  s->ia = s->cur;
  s->ib = s->ix = s->bt;
  s->io = s->bw;
  s->c2 = a;
  s->c1 = -(a * xs);
  s->c0 = xs;
}

__device__ void finish(SnfState* s, int status) {
  if ((status == SNF_OK || status == SNF_OK_FLOOR) && s->has_nocc) {
    const double err = s->t1 - (double)s->n_occ;
    if (fabs(err) >= 0.5) status = SNF_EMIXED;
  }
  s->status = status;
  s->stop = 1;
}

// The scalar state machine, run by one thread on a copy of the state's header in LDS (s);
// the per-iteration log record goes straight to the state in device memory (sg; not written
// when sg is null).
__device__ void schedule_step(SnfState* __restrict__ s, SnfState* __restrict__ sg, double e2,
                              double t1, double t2, int init) {
  if (init) {
    s->t1 = t1;
    s->t2 = t2;
    decide(s);
    return;
  }
  s->products += 1;
  if (s->prec == kPrecF64) s->products_f64 += 1; else s->products_lowp += 1;
  if (s->kind == kKindSquare) {
    const double e = sqrt(e2);
    s->e_last = e;
    const int it = s->iter;
    snf_log_rec dummy;
    snf_log_rec* rec = sg ? &sg->log[it < SNF_LOG_MAX ? it : SNF_LOG_MAX - 1] : &dummy;
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
    if (s->pmm_m) {
      pmm_next(s);
      return;
    }
    if (s->pij_i) {
      pij_next(s);
      return;
    }
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
  } else if (s->kind == kKindHorner) {
    s->horner_left -= 1;
    if (s->pij_i) pij_next(s); else pmm_next(s);
  } else {                                  // kKindCube or kKindFinal: X_new is complete
    advance_beta(s, s->branch, s->alpha);
    s->iter += 1;
    s->cur = s->io;
    s->t1 = t1;
    s->t2 = t2;
    decide(s);
  }
}

// Reduce the partial sums in a fixed order, then advance the scalar state.  The state's
// header (everything before the log) is staged in LDS by all threads, advanced there by
// thread 0 and written back by all threads: one pass of coalesced accesses instead of a
// chain of dependent single-thread loads and stores to device memory.
constexpr int kStateHeaderBytes = (int)offsetof(SnfState, log);

__device__ void schedule_body(SnfState* __restrict__ sg, const double* __restrict__ partials,
                              int count, int init) {
  __shared__ double red[24];
  __shared__ __attribute__((aligned(16))) SnfState hs;   // only the header is used
  unsigned char* hb = (unsigned char*)&hs;
  const unsigned char* gb = (const unsigned char*)sg;
  for (int i = threadIdx.x; i < kStateHeaderBytes; i += kReduceThreads) hb[i] = gb[i];
  double e2 = 0.0, t1 = 0.0, t2 = 0.0;
  for (int i = threadIdx.x; i < count; i += kReduceThreads) {
    e2 += partials[i * 4 + 0];
    t1 += partials[i * 4 + 1];
    t2 += partials[i * 4 + 2];
  }
  block_sum3(e2, t1, t2, red);             // its barrier also publishes the header copy
  if (threadIdx.x == 0) schedule_step(&hs, sg, e2, t1, t2, init);
  __syncthreads();
  unsigned char* gw = (unsigned char*)sg;
  for (int i = threadIdx.x; i < kStateHeaderBytes; i += kReduceThreads) gw[i] = hb[i];
}

// ---------------------------------------------------------------------------------------
// Small orders, whole solve in one cooperative launch: every workgroup owns one 32x32 tile
// and a private LDS copy of the scalar state.  A step is the tile product, one grid barrier,
// then every workgroup reduces all tiles' partial sums in the same fixed order and advances
// its own copy of the state: identical inputs and code give identical states, so all
// workgroups agree on the next product and on when to stop without a second barrier
// (workgroup 0 also writes the log and, at the end, the state).  Partial sums alternate
// between two buffers by step parity, so a step's sums are not overwritten before every
// workgroup has read them.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kSmallThreads) void solve_small_kernel(SnfState* __restrict__ sg,
                                                                    const Buffers* __restrict__ bufs,
                                                                    SmallGrid g,
                                                                    double* __restrict__ partials2,
                                                                    int max_steps) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  __shared__ double part[4][kSmallTile][kSmallTile + 1];
  __shared__ double red[24];
  __shared__ __attribute__((aligned(16))) SnfState hs;   // only the header is used
  unsigned char* hb = (unsigned char*)&hs;
  const unsigned char* gb = (const unsigned char*)sg;
  for (int i = threadIdx.x; i < kStateHeaderBytes; i += kSmallThreads) hb[i] = gb[i];
  __syncthreads();
  SnfState* log_to = blockIdx.x == 0 ? sg : nullptr;
  for (int step = 0; step < max_steps; ++step) {
    if (hs.stop) break;                     // the same decision in every workgroup
    double* pbuf = partials2 + (size_t)(step & 1) * g.tiles * 4;
    small_tile_product(&hs, bufs, g, blockIdx.x, pbuf, part);
    grid.sync();
    double e2 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int i = threadIdx.x; i < g.tiles; i += kSmallThreads) {
      e2 += pbuf[i * 4 + 0];
      t1 += pbuf[i * 4 + 1];
      t2 += pbuf[i * 4 + 2];
    }
    block_sum3(e2, t1, t2, red);
    if (threadIdx.x == 0) schedule_step(&hs, log_to, e2, t1, t2, 0);
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    unsigned char* gw = (unsigned char*)sg;
    for (int i = threadIdx.x; i < kStateHeaderBytes; i += kSmallThreads) gw[i] = hb[i];
  }
}

int launch_solve_small(SnfState* st, const Buffers* bufs_dev, const SmallGrid& g,
                       double* partials2, int max_steps, hipStream_t s) {
  void* args[] = {(void*)&st, (void*)&bufs_dev, (void*)&g, (void*)&partials2, (void*)&max_steps};
  return hipLaunchCooperativeKernel((const void*)solve_small_kernel, dim3(g.tiles),
                                    dim3(kSmallThreads), args, 0, s) == hipSuccess
             ? 0
             : -1;
}

__global__ __launch_bounds__(kReduceThreads) void schedule_kernel(SnfState* __restrict__ s,
                                                                  const double* __restrict__ partials,
                                                                  int count, int init) {
  if (s->stop) return;
  schedule_body(s, partials, count, init);
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
  __shared__ double red[24];
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

// ---------------------------------------------------------------------------------------
// Subspace correction (one Newton step on the occupied subspace that re-references F): the
// elementwise parts.  Every kernel walks 32 x 32 tiles of the padded order with a grid-stride
// loop; a tile's transposed partner is staged through LDS so that both reads are coalesced.
// Entries outside the true order n are written as 0, like every other padded buffer.
// ---------------------------------------------------------------------------------------
// V = W + W^T - 2 M (the coupling of G between the subspace of D~ and its complement, with
// W = G D~ and M = D~ G D~), X1 = V, Xbd = G - V (G's part that commutes with D~).
__global__ __launch_bounds__(256) void newton_split_kernel(const double* __restrict__ G,
                                                           const double* __restrict__ W,
                                                           const double* __restrict__ M,
                                                           int64_t n, int64_t np,
                                                           double* __restrict__ Xbd,
                                                           float* __restrict__ Xbd_lp,
                                                           double* __restrict__ X1,
                                                           float* __restrict__ X1_lp) {
  __shared__ double wt[32][33];
  const int64_t nt = np / 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int64_t t = blockIdx.x; t < nt * nt; t += gridDim.x) {
    const int64_t bi = t / nt, bj = t % nt;
    __syncthreads();
    for (int r = ty; r < 32; r += 8) wt[r][tx] = W[(bj * 32 + r) * np + bi * 32 + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int64_t gr = bi * 32 + r, gc = bj * 32 + tx;
      const int64_t idx = gr * np + gc;
      double v = (W[idx] + wt[tx][r]) - 2.0 * M[idx];
      double xb = G[idx] - v;
      if (gr >= n || gc >= n) v = xb = 0.0;
      X1[idx] = v;
      Xbd[idx] = xb;
      if (X1_lp) X1_lp[idx] = (float)v;
      if (Xbd_lp) Xbd_lp[idx] = (float)xb;
    }
  }
}

// X1_new = c2 (Z + Z^T) + c1 X1: the derivative of the step X <- c2 X^2 + c1 X + c0 I along
// X1, with Z = X X1 (so Z^T = X1 X for symmetric X and X1).  Exactly symmetric.
__global__ __launch_bounds__(256) void newton_sym_kernel(const double* __restrict__ Z,
                                                         const double* __restrict__ X1,
                                                         double c2, double c1, int64_t n,
                                                         int64_t np, double* __restrict__ out,
                                                         float* __restrict__ out_lp) {
  __shared__ double zt[32][33];
  const int64_t nt = np / 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int64_t t = blockIdx.x; t < nt * nt; t += gridDim.x) {
    const int64_t bi = t / nt, bj = t % nt;
    __syncthreads();
    for (int r = ty; r < 32; r += 8) zt[r][tx] = Z[(bj * 32 + r) * np + bi * 32 + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int64_t gr = bi * 32 + r, gc = bj * 32 + tx;
      const int64_t idx = gr * np + gc;
      double y = c2 * (Z[idx] + zt[tx][r]) + c1 * X1[idx];
      if (gr >= n || gc >= n) y = 0.0;
      out[idx] = y;
      if (out_lp) out_lp[idx] = (float)y;
    }
  }
}

// out = D~ + X1 (the first-order corrected projector) and per-block FP64 sums of its trace
// and squared Frobenius norm, in the partial-sum layout of f0_kernel (the refinement's
// schedule starts from them).
__global__ __launch_bounds__(256) void newton_add_kernel(const double* __restrict__ Dt,
                                                         const double* __restrict__ X1,
                                                         int64_t n, int64_t np,
                                                         double* __restrict__ out,
                                                         double* __restrict__ partials) {
  __shared__ double red[24];
  double t1 = 0.0, t2 = 0.0;
  const int64_t total = np * np;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / np, c = idx % np;
    double y = Dt[idx] + X1[idx];
    if (r >= n || c >= n) y = 0.0;
    out[idx] = y;
    if (r == c) t1 += y;
    t2 += y * y;
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

// Write the operand / output indices, precision and epilogue coefficients of the next product
// of a host-planned sequence into the state the product kernels read.
__global__ void newton_set_kernel(SnfState* __restrict__ st, const NewtonOp* __restrict__ ops,
                                  int k) {
  if (threadIdx.x != 0) return;
  const NewtonOp o = ops[k];
  st->ia = o.ia;
  st->ib = o.ib;
  st->ix = o.ix;
  st->io = o.io;
  st->prec = o.prec;
  st->write_lowp = o.write_lowp;
  st->c2 = o.c2;
  st->c1 = o.c1;
  st->c0 = o.c0;
  st->want_e = 0;
  st->dual = 0;
  st->stop = 0;
}

void launch_newton_split(const double* G, const double* W, const double* M, int64_t n,
                         int64_t np, double* Xbd, float* Xbd_lp, double* X1, float* X1_lp,
                         hipStream_t s) {
  hipLaunchKernelGGL(newton_split_kernel, dim3(kF0Blocks), dim3(256), 0, s, G, W, M, n, np, Xbd,
                     Xbd_lp, X1, X1_lp);
}

void launch_newton_sym(const double* Z, const double* X1, double c2, double c1, int64_t n,
                       int64_t np, double* out, float* out_lp, hipStream_t s) {
  hipLaunchKernelGGL(newton_sym_kernel, dim3(kF0Blocks), dim3(256), 0, s, Z, X1, c2, c1, n, np,
                     out, out_lp);
}

void launch_newton_add(const double* Dt, const double* X1, int64_t n, int64_t np, double* out,
                       double* partials, hipStream_t s) {
  hipLaunchKernelGGL(newton_add_kernel, dim3(kF0Blocks), dim3(256), 0, s, Dt, X1, n, np, out,
                     partials);
}

void launch_newton_set(SnfState* st, const NewtonOp* ops, int k, hipStream_t s) {
  hipLaunchKernelGGL(newton_set_kernel, dim3(1), dim3(64), 0, s, st, ops, k);
}

// ---------------------------------------------------------------------------------------
// Grouped launches over many independent purifications (the serving loop): workgroup b of
// a launch belongs to active request a with offs[a] <= b < offs[a+1] and computes whole
// tile b - offs[a] of that request's pending product, exactly as the single-request
// kernels do (same decomposition, same partial-sum slots), so a request's results do not
// depend on which other requests share the launch.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int group_find(const int* __restrict__ offs, int nactive, int b) {
  int lo = 0, hi = nactive;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offs[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ ProductGrid slot_grid(const SlotDesc& sd) {
  ProductGrid g;
  g.np = sd.np;
  g.n = sd.n;
  g.sym = 1;
  g.dp_tiles = num_product_tiles_dev(sd.np);
  g.tail_tiles = 0;
  g.split_s = 1;
  g.partial_count = g.dp_tiles;
  g.partials = sd.partials;
  g.split_buf = nullptr;
  return g;
}

// DUAL: the FP64 variant whose epilogue also writes the second output (the first product of
// a P_{i,j} iteration); each request's state selects exactly one of the two FP64 variants.
template <typename T, int PREC, bool DUAL = false>
__global__ __launch_bounds__(Layout<T>::NT, 2) void grouped_product_kernel(const SlotDesc* __restrict__ slots,
                                                                 const int* __restrict__ active,
                                                                 const int* __restrict__ offs,
                                                                 int nactive) {
  const int a = group_find(offs, nactive, blockIdx.x);
  const SlotDesc sd = slots[active[a]];
  if (sd.st->stop || sd.st->prec != PREC || (PREC == kPrecF64 && (sd.st->dual != 0) != DUAL))
    return;
  const ProductGrid g = slot_grid(sd);
  WorkItem wi;
  wi.tile = blockIdx.x - offs[a];
  wi.piece = -1;
  wi.kt_begin = 0;
  wi.kt_end = (int)(sd.np / Mfma<T>::kBK);
  product_body<T, PREC, DUAL>(sd.st, sd.bufs, g, wi);
}

__global__ __launch_bounds__(256, 2) void grouped_product_bf16_kernel(const SlotDesc* __restrict__ slots,
                                                                      const int* __restrict__ active,
                                                                      const int* __restrict__ offs,
                                                                      int nactive) {
  const int a = group_find(offs, nactive, blockIdx.x);
  const SlotDesc sd = slots[active[a]];
  if (sd.st->stop || sd.st->prec != kPrecBF16) return;
  const ProductGrid g = slot_grid(sd);
  WorkItem wi;
  wi.tile = blockIdx.x - offs[a];
  wi.piece = -1;
  wi.kt_begin = 0;
  wi.kt_end = (int)(sd.np / 64);
  product_bf16_body(sd.st, sd.bufs, g, wi);
}

__global__ __launch_bounds__(kReduceThreads) void grouped_schedule_kernel(const SlotDesc* __restrict__ slots,
                                                                          const int* __restrict__ active) {
  const SlotDesc sd = slots[active[blockIdx.x]];
  if (sd.st->stop) return;
  schedule_body(sd.st, sd.partials, num_product_tiles_dev(sd.np), 0);
}

__global__ void grouped_stop_kernel(const SlotDesc* __restrict__ slots, const int* __restrict__ active,
                                    int nactive, int32_t* __restrict__ stop_out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  // 0 while running; once stopped, 1 + the index of the buffer holding the result
  if (a < nactive) {
    const SnfState* st = slots[active[a]].st;
    stop_out[a] = st->stop ? 1 + st->cur : 0;
  }
}

void launch_grouped_step(int prec_mask, const SlotDesc* slots, const int* active,
                         const int* offs, int nactive, int total_tiles, int32_t* stop_out,
                         hipStream_t s, hipStream_t s2, hipEvent_t fork, hipEvent_t join) {
  if (nactive <= 0) return;
  const bool lowp = (prec_mask & ((1 << kPrecF32) | (1 << kPrecBF16))) != 0;
  // the low-precision launch goes to s2 after everything on s so far, and s waits for it
  // before the schedule: the two product grids (different requests) share the GPU
  const bool split = lowp && s2 && fork && join &&
                     hipEventRecord(fork, s) == hipSuccess &&
                     hipStreamWaitEvent(s2, fork, 0) == hipSuccess;
  hipStream_t sl = split ? s2 : s;
  if (prec_mask & (1 << kPrecF32))
    hipLaunchKernelGGL((grouped_product_kernel<float, kPrecF32>), dim3(total_tiles),
                       dim3(Layout<float>::NT), 0, sl, slots, active, offs, nactive);
  if (prec_mask & (1 << kPrecBF16))
    hipLaunchKernelGGL(grouped_product_bf16_kernel, dim3(total_tiles), dim3(kThreads), 0, sl,
                       slots, active, offs, nactive);
  if (prec_mask & (1 << kPrecF64))
    hipLaunchKernelGGL((grouped_product_kernel<double, kPrecF64>), dim3(total_tiles),
                       dim3(Layout<double>::NT), 0, s, slots, active, offs, nactive);
  if (prec_mask & kGroupedDualBit)
    hipLaunchKernelGGL((grouped_product_kernel<double, kPrecF64, true>), dim3(total_tiles),
                       dim3(Layout<double>::NT), 0, s, slots, active, offs, nactive);
  if (split && (hipEventRecord(join, s2) != hipSuccess ||
                hipStreamWaitEvent(s, join, 0) != hipSuccess))
    (void)hipStreamSynchronize(s2);    // the schedule must not start before that product
  hipLaunchKernelGGL(grouped_schedule_kernel, dim3(nactive), dim3(kReduceThreads), 0, s, slots,
                     active);
  hipLaunchKernelGGL(grouped_stop_kernel, dim3((nactive + 255) / 256), dim3(256), 0, s, slots,
                     active, nactive, stop_out);
}

}  // namespace snf
