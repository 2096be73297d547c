// Bounds of the spectrum and of the gap edges, the inputs both algorithms take (the bounds
// paragraph after Fig. 3: extremal eigenvalues or bounds thereof, and for the scaled
// varying-mu scheme a lower bound of the highest occupied and an upper bound of the lowest
// unoccupied eigenvalue, obtainable from methods for interior eigenvalues).
//
// Lanczos with full reorthogonalisation runs on the device: the symmetric matrix-vector
// product reads only the upper triangle of the matrix in 64x64 tiles (row part and
// transposed column part of each off-diagonal tile from one LDS copy; HBM-bound, one pass over
// half the matrix per product), the Gram-Schmidt passes are fixed-order reductions, so every
// run gives the same tridiagonal bit for bit.  The host diagonalises the small tridiagonal
// (cyclic Jacobi) and forms the bounds.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/snf.h"

namespace snf {
namespace {

constexpr int kT = 64;              // tile side of the matrix-vector product
constexpr int kMaxSteps = 512;
constexpr int kVecThreads = 256;
constexpr double kBreakdown = 1e-12;

#define BD_HIP(call)                                    \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) {                             \
      (void)hipGetLastError();                          \
      return SNF_EDEVICE;                               \
    }                                                   \
  } while (0)

// ---- symmetric matrix-vector product from the upper triangle ---------------------------
// Up to two vectors share each read of the matrix: y_v = a_v (M x_v) + b_v x_v.
struct SymvArgs {
  const double* M;
  int64_t ld, n, np;
  int nv;
  int abs_mode;                 // 1: use |M| (Gershgorin row sums)
  const double* x[2];
  double* y[2];
  double a[2], b[2];
  double* part;                 // [nt][nt][nv][2 kT]: row part, then column part
};

// One workgroup per upper tile (I, J), I <= J: the tile goes to LDS once; the row part
// M_IJ x_J (for block I) and, off the diagonal, the column part M_IJ^T x_I (for block J).
// A diagonal tile holds only its upper triangle in memory and is mirrored in LDS.
__global__ __launch_bounds__(256) void symv_tile_kernel(SymvArgs g, int nt) {
  const int J = blockIdx.x, I = blockIdx.y;
  if (I > J) return;
  __shared__ double tile[kT][kT + 1];
  __shared__ double xs[2][2][kT];          // [vector][I or J][k]
  constexpr int kPer = kT * kT / 256;      // values per thread
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)I * kT, c0 = (int64_t)J * kT;
  double ld[kPer];                         // all loads in flight before the first LDS store
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int idx = e * 256 + t, r = idx / kT, c = idx % kT;
    ld[e] = (r0 + r < g.n && c0 + c < g.n && (I != J || c >= r))
                ? g.M[(r0 + r) * g.ld + c0 + c] : 0.0;
  }
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int idx = e * 256 + t, r = idx / kT, c = idx % kT;
    tile[r][c] = g.abs_mode ? fabs(ld[e]) : ld[e];
  }
  if (t < 2 * kT) {
    const int which = t / kT, k = t % kT;
    for (int v = 0; v < g.nv; ++v) xs[v][which][k] = g.x[v][(which ? c0 : r0) + k];
  }
  __syncthreads();
  if (I == J) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = e * 256 + t, r = idx / kT, c = idx % kT;
      if (r > c) tile[r][c] = tile[c][r];
    }
    __syncthreads();
  }
  const int v = t / (2 * kT), rem = t % (2 * kT);
  if (v >= g.nv) return;
  double* out = g.part + (((size_t)I * nt + J) * g.nv + v) * (2 * kT);
  if (rem < kT) {                           // row part, row rem of block I
    double s = 0.0;
    for (int c = 0; c < kT; ++c) s += tile[rem][c] * xs[v][1][c];
    out[rem] = s;
  } else if (I != J) {                      // column part, column rem - kT of block J
    const int c = rem - kT;
    double s = 0.0;
    for (int r = 0; r < kT; ++r) s += tile[r][c] * xs[v][0][r];
    out[rem] = s;
  }
}

// y_v[i] = a_v (sum of the row parts of tiles (B, J >= B) and the column parts of tiles
// (I < B, B)) + b_v x_v[i]; zero beyond n.  One workgroup per row block B and vector: 16
// groups of 64 threads each take every 16th tile, then the 16 partial sums of a row are
// added in group order (fixed order, no atomics).
__global__ __launch_bounds__(1024) void symv_reduce_kernel(SymvArgs g, int nt) {
  __shared__ double acc[16][kT];
  const int B = blockIdx.x, v = blockIdx.y;
  const int grp = threadIdx.x / kT, r = threadIdx.x % kT;
  double s = 0.0;
  // tiles of block row B in the order J = B..nt-1, then I = 0..B-1 (column parts)
  for (int q = grp; q < nt; q += 16) {
    if (q < nt - B) {
      const int J = B + q;
      s += g.part[(((size_t)B * nt + J) * g.nv + v) * (2 * kT) + r];
    } else {
      const int I = q - (nt - B);
      s += g.part[(((size_t)I * nt + B) * g.nv + v) * (2 * kT) + kT + r];
    }
  }
  acc[grp][r] = s;
  __syncthreads();
  if (grp != 0) return;
  double tot = 0.0;
  for (int k = 0; k < 16; ++k) tot += acc[k][r];
  const int64_t i = (int64_t)B * kT + r;
  g.y[v][i] = i < g.n ? g.a[v] * tot + g.b[v] * g.x[v][i] : 0.0;
}

// d[i] = M[i][i] for i < n.
__global__ __launch_bounds__(256) void diag_kernel(const double* M, int64_t ld, int64_t n,
                                                   double* d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = M[i * ld + i];
}

// ---- Lanczos vector operations (chains along blockIdx.y) -------------------------------
struct Chains {
  double* V;       // [chain][kMax + 1][np]
  double* w;       // [chain][np]
  double* h;       // [chain][kMax + 1]
  double* alpha;   // [chain][kMax]
  double* beta;    // [chain][kMax]
  int64_t np;
  int kmax;
};

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kVecThreads / 64; ++k) s += red[k];
  return s;                     // valid in thread 0
}

// h_k = V_k . w for k <= j; the pass's h_j goes into alpha_j (set on pass 0, added on 1).
__global__ __launch_bounds__(kVecThreads) void lz_dots_kernel(Chains c, int j, int pass) {
  __shared__ double red[kVecThreads / 64];
  const int k = blockIdx.x, ch = blockIdx.y;
  const double* Vk = c.V + ((size_t)ch * (c.kmax + 1) + k) * c.np;
  const double* w = c.w + (size_t)ch * c.np;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < c.np; i += kVecThreads) s += Vk[i] * w[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    c.h[(size_t)ch * (c.kmax + 1) + k] = s;
    if (k == j) {
      double* a = c.alpha + (size_t)ch * c.kmax + j;
      *a = pass == 0 ? s : *a + s;
    }
  }
}

// w <- w - sum_{k <= j} h_k V_k, the sum in increasing k for every element.
__global__ __launch_bounds__(kVecThreads) void lz_update_kernel(Chains c, int j) {
  const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  const int ch = blockIdx.y;
  if (i >= c.np) return;
  const double* V = c.V + (size_t)ch * (c.kmax + 1) * c.np;
  const double* h = c.h + (size_t)ch * (c.kmax + 1);
  double acc = 0.0;
#pragma unroll 8
  for (int k = 0; k <= j; ++k) acc += h[k] * V[(size_t)k * c.np + i];
  c.w[(size_t)ch * c.np + i] -= acc;
}

// out[ch * ostride] = ||x_ch|| (one workgroup per chain, fixed order).
__global__ __launch_bounds__(1024) void lz_norm_kernel(const double* x, int64_t xstride,
                                                       double* out, int64_t ostride,
                                                       int64_t np) {
  __shared__ double red[16];
  const int ch = blockIdx.y;
  const double* v = x + (size_t)ch * xstride;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += 1024) s += v[i] * v[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tsum = 0.0;
    for (int k = 0; k < 16; ++k) tsum += red[k];
    out[(size_t)ch * ostride] = sqrt(tsum);
  }
}

// dst_ch = x_ch / nrm_ch (a zero norm leaves zeros: a breakdown, where T is cut).
__global__ __launch_bounds__(kVecThreads) void lz_scale_kernel(const double* x, int64_t xstride,
                                                               const double* nrm,
                                                               int64_t nstride, double* dst,
                                                               int64_t dstride, int64_t np) {
  const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  const int ch = blockIdx.y;
  if (i >= np) return;
  const double b = nrm[(size_t)ch * nstride];
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  dst[(size_t)ch * dstride + i] = x[(size_t)ch * xstride + i] * inv;
}

// x = 1 on [0, n), 0 beyond.
__global__ __launch_bounds__(kVecThreads) void fill_ones_kernel(double* x, int64_t n,
                                                                int64_t np) {
  const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (i < np) x[i] = i < n ? 1.0 : 0.0;
}

// V_0 = s / ||s|| for every chain; s = start (n values, zero padded), or the fixed
// pseudo-random vector u_i in [-1, 1) from SplitMix64 of i (Steele, Lea, Flood 2014).
__device__ __forceinline__ double splitmix_uniform(uint64_t i) {
  uint64_t z = i + 0x9E3779B97F4A7C15ull * (i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(kVecThreads) void lz_start_kernel(Chains c, const double* start,
                                                               int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  const int ch = blockIdx.y;
  if (i >= c.np) return;
  double v = 0.0;
  if (i < n) v = start ? start[i] : splitmix_uniform((uint64_t)i);
  c.w[(size_t)ch * c.np + i] = v;
}

// ---- host side -------------------------------------------------------------------------

// Eigenvalues and last eigenvector components of the symmetric tridiagonal (a, b) of order
// k by cyclic Jacobi rotations on the dense k x k matrix.
static void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, int k,
                             double* tmin, double* smin_last, double* tmax,
                             double* smax_last) {
  std::vector<double> A((size_t)k * k, 0.0), Q((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) {
    A[(size_t)i * k + i] = a[i];
    Q[(size_t)i * k + i] = 1.0;
    if (i + 1 < k) A[(size_t)i * k + i + 1] = A[(size_t)(i + 1) * k + i] = b[i];
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int p = 0; p < k; ++p)
      for (int q = 0; q < k; ++q) {
        const double v = A[(size_t)p * k + q] * A[(size_t)p * k + q];
        tot += v;
        if (p != q) off += v;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[(size_t)p * k + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int r = 0; r < k; ++r) {          // columns p, q
          const double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
          A[(size_t)r * k + p] = cs * arp - sn * arq;
          A[(size_t)r * k + q] = sn * arp + cs * arq;
        }
        for (int r = 0; r < k; ++r) {          // rows p, q
          const double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
          A[(size_t)p * k + r] = cs * apr - sn * aqr;
          A[(size_t)q * k + r] = sn * apr + cs * aqr;
        }
        for (int r = 0; r < k; ++r) {          // eigenvectors (columns of Q)
          const double qrp = Q[(size_t)r * k + p], qrq = Q[(size_t)r * k + q];
          Q[(size_t)r * k + p] = cs * qrp - sn * qrq;
          Q[(size_t)r * k + q] = sn * qrp + cs * qrq;
        }
      }
  }
  int imin = 0, imax = 0;
  for (int i = 1; i < k; ++i) {
    if (A[(size_t)i * k + i] < A[(size_t)imin * k + imin]) imin = i;
    if (A[(size_t)i * k + i] > A[(size_t)imax * k + imax]) imax = i;
  }
  *tmin = A[(size_t)imin * k + imin];
  *tmax = A[(size_t)imax * k + imax];
  *smin_last = fabs(Q[(size_t)(k - 1) * k + imin]);
  *smax_last = fabs(Q[(size_t)(k - 1) * k + imax]);
}

// (theta_min, r_min, theta_max, r_max) from the Lanczos coefficients: T cut at the first
// beta_j <= 1e-12 max |alpha_0..j| (then the residuals are zero).
static void ritz_from(const double* al, const double* be, int steps, double* out4) {
  int k = steps;
  bool broke = false;
  double amax = 0.0;
  for (int j = 0; j < steps; ++j) {
    amax = std::max(amax, fabs(al[j]));
    if (be[j] <= kBreakdown * amax) {
      k = j + 1;
      broke = true;
      break;
    }
  }
  std::vector<double> a(al, al + k), b(be, be + k);
  double tmin, smin, tmax, smax;
  tridiag_extremes(a, b, k, &tmin, &smin, &tmax, &smax);
  const double tail = broke ? 0.0 : b[k - 1];
  out4[0] = tmin;
  out4[1] = tail * smin;
  out4[2] = tmax;
  out4[3] = tail * smax;
}

struct BoundsWorkspace {
  int64_t np = 0;
  int kmax = 0, nv = 0;
  double *V = nullptr, *w = nullptr, *h = nullptr, *alpha = nullptr, *beta = nullptr;
  double *y = nullptr, *z = nullptr, *part = nullptr;
  double* s0 = nullptr;         // [chain] norm of the start vector
  double* host = nullptr;       // pinned read-back
  size_t host_cap = 0;
  std::mutex mu;
};

static std::mutex g_bd_mu;
static BoundsWorkspace* g_bd[64];

static BoundsWorkspace* bounds_workspace() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(g_bd_mu);
  if (!g_bd[dev]) g_bd[dev] = new BoundsWorkspace();
  return g_bd[dev];
}

static void release(BoundsWorkspace* w) {
  double** ptrs[] = {&w->V, &w->w, &w->h, &w->alpha, &w->beta, &w->y, &w->z, &w->part,
                     &w->s0};
  for (double** p : ptrs) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  w->np = 0;
  w->kmax = 0;
  w->nv = 0;
}

static int ensure(BoundsWorkspace* w, int64_t np, int kmax, int nv) {
  if (np > w->np || kmax > w->kmax || nv > w->nv) {
    release(w);
    const int nt = (int)(np / kT);
    const size_t sizes[] = {(size_t)nv * (kmax + 1) * np, (size_t)nv * np,
                            (size_t)nv * (kmax + 1), (size_t)nv * kmax, (size_t)nv * kmax,
                            (size_t)nv * np, (size_t)nv * np,
                            (size_t)nt * nt * nv * 2 * kT, (size_t)nv};
    double** ptrs[] = {&w->V, &w->w, &w->h, &w->alpha, &w->beta, &w->y, &w->z, &w->part,
                       &w->s0};
    for (int i = 0; i < 9; ++i)
      if (hipMalloc(ptrs[i], sizes[i] * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        release(w);
        return SNF_ENOMEM;
      }
    w->np = np;
    w->kmax = kmax;
    w->nv = nv;
  }
  const size_t need = (size_t)2 * nv * kmax + 2 * (size_t)np;
  if (need > w->host_cap) {
    if (w->host) (void)hipHostFree(w->host);
    w->host = nullptr;
    w->host_cap = 0;
    BD_HIP(hipHostMalloc(&w->host, need * sizeof(double), hipHostMallocDefault));
    w->host_cap = need;
  }
  return SNF_OK;
}

static void launch_symv(const SymvArgs& g, hipStream_t s) {
  const int nt = (int)(g.np / kT);
  hipLaunchKernelGGL(symv_tile_kernel, dim3(nt, nt), dim3(256), 0, s, g, nt);
  hipLaunchKernelGGL(symv_reduce_kernel, dim3(nt, g.nv), dim3(1024), 0, s, g, nt);
}

static SymvArgs symv_args(const double* M, int64_t ld, int64_t n, int64_t np, int nv,
                          double* part) {
  SymvArgs g;
  memset(&g, 0, sizeof(g));
  g.M = M;
  g.ld = ld;
  g.n = n;
  g.np = np;
  g.nv = nv;
  g.part = part;
  return g;
}

// Lanczos on nv chains; apply(j) must leave A v_j of every chain in c.w.
template <typename Apply>
static int run_lanczos(BoundsWorkspace* w, int64_t n, int64_t np, int nv, int steps,
                       const double* start, Apply apply, hipStream_t s) {
  Chains c{w->V, w->w, w->h, w->alpha, w->beta, np, w->kmax};
  const int64_t vstride = (int64_t)(c.kmax + 1) * np;
  const dim3 gv((unsigned)((np + kVecThreads - 1) / kVecThreads), nv);
  hipLaunchKernelGGL(lz_start_kernel, gv, dim3(kVecThreads), 0, s, c, start, n);
  hipLaunchKernelGGL(lz_norm_kernel, dim3(1, nv), dim3(1024), 0, s, c.w, np, w->s0,
                     (int64_t)1, np);
  hipLaunchKernelGGL(lz_scale_kernel, gv, dim3(kVecThreads), 0, s, c.w, np, w->s0, (int64_t)1,
                     c.V, vstride, np);
  BD_HIP(hipGetLastError());
  for (int j = 0; j < steps; ++j) {
    apply(j);
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(lz_dots_kernel, dim3(j + 1, nv), dim3(kVecThreads), 0, s, c, j, pass);
      hipLaunchKernelGGL(lz_update_kernel, gv, dim3(kVecThreads), 0, s, c, j);
    }
    hipLaunchKernelGGL(lz_norm_kernel, dim3(1, nv), dim3(1024), 0, s, c.w, np, c.beta + j,
                       (int64_t)c.kmax, np);
    hipLaunchKernelGGL(lz_scale_kernel, gv, dim3(kVecThreads), 0, s, c.w, np, c.beta + j,
                       (int64_t)c.kmax, c.V + (size_t)(j + 1) * np, vstride, np);
    BD_HIP(hipGetLastError());
  }
  return SNF_OK;
}

}  // namespace

void bounds_release_all_devices() {
  int prev = 0;
  const bool restore = hipGetDevice(&prev) == hipSuccess;
  for (int dev = 0; dev < 64; ++dev) {
    BoundsWorkspace* w = nullptr;
    {
      std::lock_guard<std::mutex> g(g_bd_mu);
      w = g_bd[dev];
    }
    if (!w || hipSetDevice(dev) != hipSuccess) continue;
    std::lock_guard<std::mutex> g(w->mu);
    (void)hipDeviceSynchronize();
    release(w);
    if (w->host) (void)hipHostFree(w->host);
    w->host = nullptr;
    w->host_cap = 0;
  }
  if (restore) (void)hipSetDevice(prev);
}

}  // namespace snf

using namespace snf;

extern "C" {

int snf_spectral_bounds(const double* F_dev, int64_t n, int64_t ld, int32_t steps,
                        const double* start_dev, double* out, void* stream) {
  if (!F_dev || !out || n <= 0 || ld < n || steps < 1 || steps > kMaxSteps) return SNF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  BoundsWorkspace* w = bounds_workspace();
  if (!w) return SNF_EDEVICE;
  std::lock_guard<std::mutex> guard(w->mu);
  const int64_t np = (n + kT - 1) / kT * kT;
  int rc = ensure(w, np, std::max(steps, w->kmax), std::max(1, w->nv));
  if (rc) return rc;
  const int kmax = w->kmax;
  auto apply = [&](int j) {
    SymvArgs g = symv_args(F_dev, ld, n, np, 1, w->part);
    g.x[0] = w->V + (size_t)j * np;
    g.y[0] = w->w;
    g.a[0] = 1.0;
    g.b[0] = 0.0;
    launch_symv(g, s);
  };
  rc = run_lanczos(w, n, np, 1, steps, start_dev, apply, s);
  if (rc) return rc;
  // Gershgorin: r_i = sum_j |F_ij| from the same product with |F| and x = 1
  {
    hipLaunchKernelGGL(fill_ones_kernel, dim3((unsigned)((np + kVecThreads - 1) / kVecThreads)),
                       dim3(kVecThreads), 0, s, w->z, n, np);
    SymvArgs g = symv_args(F_dev, ld, n, np, 1, w->part);
    g.abs_mode = 1;
    g.x[0] = w->z;
    g.y[0] = w->y;
    g.a[0] = 1.0;
    g.b[0] = 0.0;
    launch_symv(g, s);
    BD_HIP(hipGetLastError());
  }
  double* hab = w->host;
  double* hrow = w->host + 2 * (size_t)w->nv * kmax;
  BD_HIP(hipMemcpyAsync(hab, w->alpha, steps * sizeof(double), hipMemcpyDeviceToHost, s));
  BD_HIP(hipMemcpyAsync(hab + kmax, w->beta, steps * sizeof(double), hipMemcpyDeviceToHost, s));
  BD_HIP(hipMemcpyAsync(hrow, w->y, n * sizeof(double), hipMemcpyDeviceToHost, s));
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, F_dev, ld,
                     n, w->z);
  BD_HIP(hipGetLastError());
  double* diag = hrow + np;
  BD_HIP(hipMemcpyAsync(diag, w->z, n * sizeof(double), hipMemcpyDeviceToHost, s));
  BD_HIP(hipStreamSynchronize(s));
  double r4[4];
  ritz_from(hab, hab + kmax, steps, r4);
  const double pad = 1e-13 * std::max(fabs(r4[0]), fabs(r4[2]));
  out[0] = r4[0] - r4[1] - pad;
  out[1] = r4[2] + r4[3] + pad;
  double glo = INFINITY, ghi = -INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    const double rad = hrow[i] - fabs(diag[i]);
    glo = std::min(glo, diag[i] - rad);
    ghi = std::max(ghi, diag[i] + rad);
  }
  out[2] = glo;
  out[3] = ghi;
  return SNF_OK;
}

int snf_gap_bounds(const double* F_dev, const double* D_dev, int64_t n, int64_t ld,
                   double lambda_min, double lambda_max, int32_t steps,
                   const double* start_dev, double* out, void* stream) {
  if (!F_dev || !D_dev || !out || n <= 0 || ld < n || steps < 1 || steps > kMaxSteps ||
      !isfinite(lambda_min) || !isfinite(lambda_max) || !(lambda_min < lambda_max))
    return SNF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  BoundsWorkspace* w = bounds_workspace();
  if (!w) return SNF_EDEVICE;
  std::lock_guard<std::mutex> guard(w->mu);
  const int64_t np = (n + kT - 1) / kT * kT;
  int rc = ensure(w, np, std::max(steps, w->kmax), 2);
  if (rc) return rc;
  const int kmax = w->kmax;
  // chain 0: D (F - lambda_min I) D;  chain 1: (I - D)(lambda_max I - F)(I - D)
  auto apply = [&](int j) {
    SymvArgs g = symv_args(D_dev, ld, n, np, 2, w->part);
    g.x[0] = w->V + (size_t)j * np;
    g.x[1] = w->V + ((size_t)(kmax + 1) + j) * np;
    g.y[0] = w->y;
    g.y[1] = w->y + np;
    g.a[0] = 1.0;  g.b[0] = 0.0;
    g.a[1] = -1.0; g.b[1] = 1.0;
    launch_symv(g, s);
    SymvArgs f = symv_args(F_dev, ld, n, np, 2, w->part);
    f.x[0] = w->y;
    f.x[1] = w->y + np;
    f.y[0] = w->z;
    f.y[1] = w->z + np;
    f.a[0] = 1.0;  f.b[0] = -lambda_min;
    f.a[1] = -1.0; f.b[1] = lambda_max;
    launch_symv(f, s);
    SymvArgs d = symv_args(D_dev, ld, n, np, 2, w->part);
    d.x[0] = w->z;
    d.x[1] = w->z + np;
    d.y[0] = w->w;
    d.y[1] = w->w + np;
    d.a[0] = 1.0;  d.b[0] = 0.0;
    d.a[1] = -1.0; d.b[1] = 1.0;
    launch_symv(d, s);
  };
  rc = run_lanczos(w, n, np, 2, steps, start_dev, apply, s);
  if (rc) return rc;
  double* hab = w->host;
  for (int ch = 0; ch < 2; ++ch) {
    BD_HIP(hipMemcpyAsync(hab + (size_t)ch * 2 * kmax, w->alpha + (size_t)ch * kmax,
                          steps * sizeof(double), hipMemcpyDeviceToHost, s));
    BD_HIP(hipMemcpyAsync(hab + (size_t)ch * 2 * kmax + kmax, w->beta + (size_t)ch * kmax,
                          steps * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  BD_HIP(hipStreamSynchronize(s));
  double r0[4], r1[4];
  ritz_from(hab, hab + kmax, steps, r0);
  ritz_from(hab + 2 * (size_t)kmax, hab + 3 * (size_t)kmax, steps, r1);
  const double pad = 1e-13 * (lambda_max - lambda_min);
  out[0] = lambda_min + r0[2] - pad;
  out[1] = lambda_max - r1[2] + pad;
  return SNF_OK;
}

}  // extern "C"
