// Streaming kernels over the tall side of an unfolding: the passes that read
// the m x n matrix A from HBM.  All accumulation is FP64; partial sums per row
// chunk are reduced in a fixed order, so results are bitwise reproducible.
#include "tt_internal.h"

namespace ttutv {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t at(int layout, int64_t i, int64_t j, int64_t m, int64_t n) {
  return layout == ROW ? i * n + j : i + j * m;
}

template <typename T>
__device__ __forceinline__ double ldv(const T* p, int64_t i) { return (double)p[i]; }

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// partials[chunk] = A[rows of chunk, j0:j0+64]^T * Y[rows of chunk, :]
// grid: (nchunks, ceil(n/64)); each thread owns a 4x4 block of the 64 x c
// output and a subset of the rows of every 32-row tile staged in LDS.
constexpr int kAtbTR = 32;
constexpr int kAtbJT = 64;

template <typename TA, typename TY>
__global__ __launch_bounds__(kThreads) void k_atb(const TA* __restrict__ A, const TY* __restrict__ Y,
                                                  int64_t m, int n, int c, int layout,
                                                  int64_t rows_per_chunk,
                                                  double* __restrict__ partials) {
  __shared__ double sA[kAtbTR][kAtbJT + 1];
  __shared__ double sY[kAtbTR][kCMax + 1];
  __shared__ double red[kThreads * 16];
  const int t = threadIdx.x;
  const int64_t chunk = blockIdx.x;
  const int j0 = blockIdx.y * kAtbJT;
  const int jt = min(kAtbJT, n - j0);
  const int nbj = (jt + 3) >> 2, nbc = (c + 3) >> 2, nblk = nbj * nbc;
  const int RG = kThreads / nblk;  // nblk <= 256, so RG >= 1
  const int blk = t % nblk, rg = t / nblk;
  const bool active = rg < RG;
  const int bj = (blk / nbc) * 4, bc = (blk % nbc) * 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;

  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = min(m, r0 + rows_per_chunk);
  for (int64_t rb = r0; rb < r1; rb += kAtbTR) {
    const int tr = (int)min((int64_t)kAtbTR, r1 - rb);
    // stage A[rb:rb+tr, j0:j0+jt] and Y[rb:rb+tr, 0:c]; zero-fill the padding
    for (int e = t; e < kAtbTR * kAtbJT; e += kThreads) {
      int i, j;
      if (layout == ROW) { i = e / kAtbJT; j = e % kAtbJT; } else { i = e % kAtbTR; j = e / kAtbTR; }
      sA[i][j] = (i < tr && j < jt) ? ldv(A, at(layout, rb + i, j0 + j, m, n)) : 0.0;
    }
    for (int e = t; e < kAtbTR * kCMax; e += kThreads) {
      int i, j;
      if (layout == ROW) { i = e / kCMax; j = e % kCMax; } else { i = e % kAtbTR; j = e / kAtbTR; }
      sY[i][j] = (i < tr && j < c) ? ldv(Y, at(layout, rb + i, j, m, c)) : 0.0;
    }
    __syncthreads();
    if (active) {
      for (int i = rg; i < tr; i += RG) {
        double a[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = sA[i][bj + u];
#pragma unroll
        for (int v = 0; v < 4; ++v) y[v] = sY[i][bc + v];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], y[v], acc[u][v]);
      }
    }
    __syncthreads();
  }
  // fixed-order reduction over the row groups
  if (active) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[(rg * nblk + blk) * 16 + u * 4 + v] = acc[u][v];
  }
  __syncthreads();
  double* out = partials + chunk * (int64_t)n * c;
  for (int e = t; e < jt * c; e += kThreads) {
    const int j = e % jt, cc = e / jt;
    const int b = (j >> 2) * nbc + (cc >> 2), u = j & 3, v = cc & 3;
    double s = 0.0;
    for (int g = 0; g < RG; ++g) s += red[(g * nblk + b) * 16 + u * 4 + v];
    out[(j0 + j) + (int64_t)n * cc] = s;
  }
}

// ---------------------------------------------------------------------------
// Y = A W.  Each thread owns a 4-row x 4-column block of the output tile of
// TR = 4 * (256 / ceil(c/4)) rows; A is staged 32 columns at a time in LDS.
constexpr int kAxKT = 32;

// Row blocks of 4 per tile: as many as the 256 threads allow, at most 64 so
// that a tile never exceeds the 256 rows staged in LDS.
__host__ __device__ __forceinline__ int ax_row_blocks(int nbc) {
  const int rb = kThreads / nbc;
  return rb < 64 ? rb : 64;
}

template <typename TA, typename TY>
__global__ __launch_bounds__(kThreads) void k_ax(const TA* __restrict__ A, const double* __restrict__ W,
                                                 TY* __restrict__ Y, int64_t m, int n, int c,
                                                 int layout, int64_t rows_per_chunk,
                                                 double* __restrict__ sumsqA,
                                                 double* __restrict__ sumsqY) {
  __shared__ double sA[kThreads][kAxKT + 1];
  __shared__ double sW[kAxKT][kCMax];
  __shared__ double sh[8];
  const int t = threadIdx.x;
  const int nbc = (c + 3) >> 2;
  const int RB = ax_row_blocks(nbc);
  const int TR = 4 * RB;  // <= kThreads rows, the height of sA
  const bool active = t < RB * nbc;
  const int bc = (t % nbc) * 4, br = (t / nbc) * 4;
  const int64_t chunk = blockIdx.x;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = min(m, r0 + rows_per_chunk);
  double ssa = 0.0, ssy = 0.0;
  for (int64_t rb = r0; rb < r1; rb += TR) {
    const int tr = (int)min((int64_t)TR, r1 - rb);
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int k0 = 0; k0 < n; k0 += kAxKT) {
      const int kt = min(kAxKT, n - k0);
      const int cnt = tr * kt;
      for (int e = t; e < cnt; e += kThreads) {
        int i, k;
        if (layout == ROW) { i = e / kt; k = e % kt; } else { i = e % tr; k = e / tr; }
        const double x = ldv(A, at(layout, rb + i, k0 + k, m, n));
        ssa = fma(x, x, ssa);
        sA[i][k] = x;
      }
      for (int e = t; e < kAxKT * kCMax; e += kThreads) {
        const int k = e % kAxKT, cc = e / kAxKT;
        sW[k][cc] = (k < kt && cc < c) ? W[(k0 + k) + (int64_t)n * cc] : 0.0;
      }
      __syncthreads();
      if (active && br < tr) {
        for (int k = 0; k < kt; ++k) {
          double a[4], w[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) a[u] = sA[min(br + u, TR - 1)][k];
#pragma unroll
          for (int v = 0; v < 4; ++v) w[v] = sW[k][bc + v];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], w[v], acc[u][v]);
        }
      }
      __syncthreads();
    }
    if (active) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (br + u >= tr) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (bc + v < c) {
            const TY y = (TY)acc[u][v];
            const double yd = (double)y;
            ssy = fma(yd, yd, ssy);
            Y[at(layout, rb + br + u, bc + v, m, c)] = y;
          }
        }
      }
    }
  }
  if (sumsqA) {
    const double s = block_sum(ssa, sh);
    if (t == 0) sumsqA[chunk] = s;
  }
  if (sumsqY) {
    const double s = block_sum(ssy, sh);
    if (t == 0) sumsqY[chunk] = s;
  }
}

// ---------------------------------------------------------------------------
// resid[chunk] = sum over rows of ||A(i,:) - Cr(i,:) V1^T||^2 (direct step error).
constexpr int kResTR = 64;

template <typename TA>
__global__ __launch_bounds__(kThreads) void k_resid(const TA* __restrict__ A, const double* __restrict__ Cr,
                                                    const double* __restrict__ V1, int64_t m, int n,
                                                    int r, int layout, int64_t rows_per_chunk,
                                                    double* __restrict__ resid) {
  __shared__ double sC[kResTR][kCMax + 1];
  __shared__ double sV[kAxKT][kCMax + 1];
  __shared__ double sh[8];
  const int t = threadIdx.x;
  const int64_t chunk = blockIdx.x;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = min(m, r0 + rows_per_chunk);
  double acc = 0.0;
  for (int64_t rb = r0; rb < r1; rb += kResTR) {
    const int tr = (int)min((int64_t)kResTR, r1 - rb);
    for (int e = t; e < tr * r; e += kThreads) {
      int i, a;
      if (layout == ROW) { i = e / r; a = e % r; } else { i = e % tr; a = e / tr; }
      sC[i][a] = Cr[at(layout, rb + i, a, m, r)];
    }
    for (int k0 = 0; k0 < n; k0 += kAxKT) {
      const int kt = min(kAxKT, n - k0);
      __syncthreads();
      for (int e = t; e < kt * r; e += kThreads) {
        const int k = e % kt, a = e / kt;
        sV[k][a] = V1[(k0 + k) + (int64_t)n * a];
      }
      __syncthreads();
      for (int e = t; e < tr * kt; e += kThreads) {
        int i, k;
        if (layout == ROW) { i = e / kt; k = e % kt; } else { i = e % tr; k = e / tr; }
        double x = ldv(A, at(layout, rb + i, k0 + k, m, n));
        for (int a = 0; a < r; ++a) x = fma(-sC[i][a], sV[k][a], x);
        acc = fma(x, x, acc);
      }
    }
    __syncthreads();
  }
  const double s = block_sum(acc, sh);
  if (t == 0) resid[chunk] = s;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_reduce(const double* __restrict__ partials, int nchunks,
                                                     int64_t size, double* __restrict__ out,
                                                     double* __restrict__ out2) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= size) return;
  double s = 0.0;
  for (int ch = 0; ch < nchunks; ++ch) s += partials[(int64_t)ch * size + e];
  out[e] = s;
  if (out2) out2[e] = s;
}

}  // namespace

// ---------------------------------------------------------------------------
int atb_chunks(int64_t m, int n, int c) {
  (void)c;
  const int64_t tiles = (m + kAtbTR - 1) / kAtbTR;
  const int colblocks = (n + kAtbJT - 1) / kAtbJT;
  int64_t want = 1024 / colblocks;
  if (want < 1) want = 1;
  return (int)(tiles < want ? tiles : want);
}

hipError_t launch_atb(const void* A, int a_f32, const void* Y, int y_f32, int64_t m, int n, int c,
                      int layout, double* partials, int nchunks, hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || m < 1 || nchunks < 1) return hipErrorInvalidValue;
  const int64_t rpc = (m + nchunks - 1) / nchunks;
  dim3 grid(nchunks, (n + kAtbJT - 1) / kAtbJT);
  if (!a_f32 && !y_f32)
    hipLaunchKernelGGL((k_atb<double, double>), grid, dim3(kThreads), 0, st, (const double*)A,
                       (const double*)Y, m, n, c, layout, rpc, partials);
  else if (a_f32 && y_f32)
    hipLaunchKernelGGL((k_atb<float, float>), grid, dim3(kThreads), 0, st, (const float*)A,
                       (const float*)Y, m, n, c, layout, rpc, partials);
  else if (a_f32)
    hipLaunchKernelGGL((k_atb<float, double>), grid, dim3(kThreads), 0, st, (const float*)A,
                       (const double*)Y, m, n, c, layout, rpc, partials);
  else
    hipLaunchKernelGGL((k_atb<double, float>), grid, dim3(kThreads), 0, st, (const double*)A,
                       (const float*)Y, m, n, c, layout, rpc, partials);
  return hipGetLastError();
}

int ax_chunks(int64_t m, int c) {
  const int nbc = (c + 3) / 4;
  const int TR = 4 * ax_row_blocks(nbc);
  const int64_t tiles = (m + TR - 1) / TR;
  return (int)(tiles < 2048 ? tiles : 2048);
}

hipError_t launch_ax(const void* A, int a_f32, const double* W, void* Y, int y_f32, int64_t m, int n,
                     int c, int layout, int nchunks, double* sumsqA, double* sumsqY,
                     hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || m < 1 || nchunks < 1) return hipErrorInvalidValue;
  const int64_t rpc = (m + nchunks - 1) / nchunks;
  dim3 grid(nchunks);
  if (!a_f32 && !y_f32)
    hipLaunchKernelGGL((k_ax<double, double>), grid, dim3(kThreads), 0, st, (const double*)A, W,
                       (double*)Y, m, n, c, layout, rpc, sumsqA, sumsqY);
  else if (a_f32 && !y_f32)
    hipLaunchKernelGGL((k_ax<float, double>), grid, dim3(kThreads), 0, st, (const float*)A, W,
                       (double*)Y, m, n, c, layout, rpc, sumsqA, sumsqY);
  else if (a_f32 && y_f32)
    hipLaunchKernelGGL((k_ax<float, float>), grid, dim3(kThreads), 0, st, (const float*)A, W,
                       (float*)Y, m, n, c, layout, rpc, sumsqA, sumsqY);
  else
    hipLaunchKernelGGL((k_ax<double, float>), grid, dim3(kThreads), 0, st, (const double*)A, W,
                       (float*)Y, m, n, c, layout, rpc, sumsqA, sumsqY);
  return hipGetLastError();
}

int resid_chunks(int64_t m) {
  const int64_t tiles = (m + kResTR - 1) / kResTR;
  return (int)(tiles < 2048 ? tiles : 2048);
}

hipError_t launch_resid(const void* A, int a_f32, const double* Cr, const double* V1, int64_t m,
                        int n, int r, int layout, int nchunks, double* resid, hipStream_t st) {
  if (n < 1 || r < 1 || r > kCMax || m < 1 || nchunks < 1) return hipErrorInvalidValue;
  const int64_t rpc = (m + nchunks - 1) / nchunks;
  if (a_f32)
    hipLaunchKernelGGL((k_resid<float>), dim3(nchunks), dim3(kThreads), 0, st, (const float*)A, Cr,
                       V1, m, n, r, layout, rpc, resid);
  else
    hipLaunchKernelGGL((k_resid<double>), dim3(nchunks), dim3(kThreads), 0, st, (const double*)A,
                       Cr, V1, m, n, r, layout, rpc, resid);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nchunks, int64_t size, double* out,
                         double* out2, hipStream_t st) {
  if (size < 1 || nchunks < 1) return hipErrorInvalidValue;
  const int64_t blocks = (size + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)blocks), dim3(kThreads), 0, st, partials, nchunks,
                     size, out, out2);
  return hipGetLastError();
}

}  // namespace ttutv
