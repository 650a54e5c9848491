// Contractions of a tensor train (Eq. (TT)): dense reconstruction as a chain
// of small-K GEMMs, entries at given multi-indices, and the gradient of a
// weighted sum of sampled entries with respect to every core.
#include <algorithm>

#include "tt_internal.h"

namespace ttutv {

namespace {

constexpr int kThreads = 256;
constexpr int TT_MAX_D_INTERNAL = 32;

// C (M x N) = A (M x K) B (K x N), column-major, K <= KB <= 64.  64 x 64
// output tile per workgroup, 4 x 4 per thread; consecutive threads own
// consecutive row quads so that the column-major writes coalesce.  The
// staged operands take about 1 KB per k (a row of 65 doubles of each), so
// KB = 16 lets eight workgroups share a CU where KB = 64 fits two: the output
// write, which bounds the kernel, needs the workgroups in flight.
template <typename TC, int KB>
__global__ __launch_bounds__(kThreads) void k_gemm_smallk(const double* __restrict__ A,
                                                          const double* __restrict__ B,
                                                          TC* __restrict__ C, int64_t M, int64_t N,
                                                          int K) {
  __shared__ double sA[KB][64 + 1];
  __shared__ double sB[KB][64 + 1];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int64_t j0 = (int64_t)blockIdx.y * 64;
  const int mi = (int)min((int64_t)64, M - i0);
  const int nj = (int)min((int64_t)64, N - j0);
  for (int e = t; e < 64 * K; e += kThreads) {
    const int i = e % 64, k = e / 64;
    sA[k][i] = (i < mi) ? A[(i0 + i) + M * k] : 0.0;
  }
  for (int e = t; e < 64 * K; e += kThreads) {
    const int k = e % K, j = e / K;
    sB[k][j] = (j < nj) ? B[k + (int64_t)K * (j0 + j)] : 0.0;
  }
  __syncthreads();
  const int ti = (t % 16) * 4, tj = (t / 16) * 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k = 0; k < K; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = sA[k][ti + u];
#pragma unroll
    for (int v = 0; v < 4; ++v) b[v] = sB[k][tj + v];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
  }
  // a full tile whose columns start 16-byte aligned: each lane's four rows of
  // a column (32 bytes of FP64, 16 of FP32) go out as 16-byte streaming stores,
  // so a wave writes whole 512-byte (256-byte) column runs per instruction and
  // the output does not displace the cached operands
  constexpr int VW = 16 / (int)sizeof(TC);   // values per 16-byte store
  const bool vec = mi == 64 && nj == 64 && (M % VW) == 0 && ((uintptr_t)C % 16) == 0;
  if (vec) {
    typedef TC vt __attribute__((ext_vector_type(VW)));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      TC* col = C + (i0 + ti) + M * (j0 + tj + v);
#pragma unroll
      for (int u0 = 0; u0 < 4; u0 += VW) {
        vt x;
#pragma unroll
        for (int q = 0; q < VW; ++q) x[q] = (TC)acc[u0 + q][v];
        __builtin_nontemporal_store(x, reinterpret_cast<vt*>(col + u0));
      }
    }
    return;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (tj + v >= nj) break;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ti + u < mi) C[(i0 + ti + u) + M * (j0 + tj + v)] = (TC)acc[u][v];
  }
}

// C (M x N, column-major) = sum over k of A(m, k) B(k, n), with A(m, k) at
// A[m sam + k sak] and B(k, n) at B[k sbk + n sbn]: any transposition of
// either operand.  Workgroup z of Z takes the k range [z kper, (z+1) kper) and
// writes its own M x N partial (out + z M N); the partials are then summed in
// a fixed order, so the result does not depend on timing.  64 x 64 output
// tile, 4 x 4 per thread, KT-deep operand tiles staged in LDS with the loads
// mapped along whichever index has unit stride.
constexpr int kGaKT = 16;

__global__ __launch_bounds__(kThreads) void k_gemm_any(const double* __restrict__ A, int64_t sam, int64_t sak,
                                                       const double* __restrict__ B, int64_t sbk, int64_t sbn,
                                                       double* __restrict__ out, int64_t M, int64_t N, int64_t K,
                                                       int64_t kper) {
  __shared__ double sA[kGaKT][64 + 1];
  __shared__ double sB[kGaKT][64 + 1];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int64_t kb = (int64_t)blockIdx.z * kper;
  const int64_t ke = min(K, kb + kper);
  const bool a_m_fast = sam <= sak, b_k_fast = sbk <= sbn;
  const int ti = (t % 16) * 4, tj = (t / 16) * 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int64_t k0 = kb; k0 < ke; k0 += kGaKT) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (64 * kGaKT) / kThreads; ++u) {
      const int e = t + kThreads * u;
      int i, k;
      if (a_m_fast) { i = e % 64; k = e / 64; } else { k = e % kGaKT; i = e / kGaKT; }
      const int64_t gi = i0 + i, gk = k0 + k;
      sA[k][i] = (gi < M && gk < ke) ? A[gi * sam + gk * sak] : 0.0;
      int j, k2;
      if (b_k_fast) { k2 = e % kGaKT; j = e / kGaKT; } else { j = e % 64; k2 = e / 64; }
      const int64_t gj = j0 + j, gk2 = k0 + k2;
      sB[k2][j] = (gj < N && gk2 < ke) ? B[gk2 * sbk + gj * sbn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kGaKT; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = sA[k][ti + u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = sB[k][tj + v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
  }
  double* C = out + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t j = j0 + tj + v;
    if (j >= N) break;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + ti + u;
      if (i < M) C[i + M * j] = acc[u][v];
    }
  }
}

// out (cols x rows, column-major) = in^T, in rows x cols column-major; 32 x 32
// tiles through LDS so that both sides are read and written along columns.
__global__ __launch_bounds__(kThreads) void k_transpose(const double* __restrict__ in, int64_t rows, int64_t cols,
                                                        double* __restrict__ out) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + tx, c = c0 + y;
    tile[y][tx] = (r < rows && c < cols) ? in[r + rows * c] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t c = c0 + tx, r = r0 + y;   // out(c, r) at c + cols r
    if (r < rows && c < cols) out[c + cols * r] = tile[tx][y];
  }
}

struct TrainDesc {
  int d;
  int64_t dims[TT_MAX_D_INTERNAL];
  int64_t ranks[TT_MAX_D_INTERNAL + 1];
  const double* cores[TT_MAX_D_INTERNAL];
};

struct GradDesc {
  double* cores[TT_MAX_D_INTERNAL];
};

__device__ __forceinline__ double core_at(const TrainDesc& D, int c, int64_t a, int64_t i, int64_t b) {
  return D.cores[c][a + D.ranks[c] * (i + D.dims[c] * b)];
}

// One wave per sample: lane b holds entry b of the running row vector
// G_1[i_1] ... G_k[i_k] (length r_k <= 64).
__global__ __launch_bounds__(kThreads) void k_sample(TrainDesc D, const int64_t* __restrict__ idx,
                                                     int64_t N, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kThreads) >> 6;
  for (int64_t s = wave; s < N; s += nwaves) {
    const int64_t* ix = idx + s * D.d;
    double v = (lane < D.ranks[1]) ? core_at(D, 0, 0, ix[0], lane) : 0.0;
    for (int c = 1; c < D.d; ++c) {
      const int ra = (int)D.ranks[c], rb = (int)D.ranks[c + 1];
      const int64_t i = ix[c];
      double nv = 0.0;
      for (int a = 0; a < ra; ++a) {
        const double va = __shfl(v, a, 64);
        if (lane < rb) nv = fma(va, core_at(D, c, a, i, lane), nv);
      }
      v = nv;
    }
    if (lane == 0) out[s] = v;
  }
}

// One wave per sample: the right interface products rho_c (c = d-1..0) are
// recomputed into LDS, then a left-to-right pass forms lambda_c and scatters
// gout_s * lambda_c[a] * rho_c[b] into dG_c[a, i_c, b].
// Left interface products from the cores of D, right ones from those of DR
// (the same train for the plain gradient; the left- and right-orthogonal
// forms of one train for the gradient at the mixed-canonical points).
__global__ __launch_bounds__(kThreads) void k_sample_bwd(TrainDesc D, TrainDesc DR, const int64_t* __restrict__ idx,
                                                         int64_t N, const double* __restrict__ gout,
                                                         GradDesc G) {
  __shared__ double rho[kThreads / 64][TT_MAX_D_INTERNAL][64];
  const int lane = threadIdx.x & 63;
  const int wl = threadIdx.x >> 6;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kThreads) >> 6;
  const int d = D.d;
  for (int64_t s = wave; s < N; s += nwaves) {
    const int64_t* ix = idx + s * d;
    const double w = gout[s];
    // rho_{d-1} = [1]; rho_c[a] = sum_b G_{c+1}[a, i_{c+1}, b] rho_{c+1}[b]
    double r = (lane == 0) ? 1.0 : 0.0;
    rho[wl][d - 1][lane] = r;
    for (int c = d - 2; c >= 0; --c) {
      const int ra = (int)D.ranks[c + 1], rb = (int)D.ranks[c + 2];
      const int64_t i = ix[c + 1];
      double nr = 0.0;
      for (int b = 0; b < rb; ++b) {
        const double rbv = __shfl(r, b, 64);
        if (lane < ra) nr = fma(core_at(DR, c + 1, lane, i, b), rbv, nr);
      }
      r = nr;
      rho[wl][c][lane] = r;
    }
    // left pass
    double l = (lane == 0) ? 1.0 : 0.0;
    for (int c = 0; c < d; ++c) {
      const int ra = (int)D.ranks[c], rb = (int)D.ranks[c + 1];
      const int64_t i = ix[c];
      const int tot = ra * rb;
      // lambda_c[a] lives in lane a; gather it by shuffle for every (a, b) entry
      for (int e0 = 0; e0 < tot; e0 += 64) {
        const int e = e0 + lane;
        const int a = (e < tot) ? e % ra : 0;
        const int b = (e < tot) ? e / ra : 0;
        const double la = __shfl(l, a, 64);
        if (e < tot) {
          const double g = w * la * rho[wl][c][b];
          atomicAdd(&G.cores[c][a + (int64_t)ra * (i + D.dims[c] * b)], g);
        }
      }
      if (c + 1 < d) {
        double nl = 0.0;
        for (int a = 0; a < ra; ++a) {
          const double la = __shfl(l, a, 64);
          if (lane < rb) nl = fma(la, core_at(D, c, a, i, lane), nl);
        }
        l = nl;
      }
    }
  }
}

__global__ void k_fill_zero(double* p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0.0;
}

bool fill_desc(TrainDesc& D, int d, const int64_t* dims, const int64_t* ranks,
               const double* const* cores) {
  if (d < 2 || d > TT_MAX_D_INTERNAL) return false;
  D.d = d;
  for (int k = 0; k < d; ++k) {
    D.dims[k] = dims[k];
    D.cores[k] = cores[k];
  }
  for (int k = 0; k <= d; ++k) D.ranks[k] = ranks[k];
  return true;
}

}  // namespace

hipError_t launch_gemm_smallk(const double* A, const double* B, void* C, int c_f32, int64_t M,
                              int64_t N, int K, hipStream_t st) {
  if (M < 1 || N < 1 || K < 1 || K > kCMax) return hipErrorInvalidValue;
  const int64_t gx = (M + 63) / 64, gy = (N + 63) / 64;
  if (gy > 65535 || gx > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)gx, (unsigned)gy);
#define TT_GSK(TCV, KBV) \
  TT_LAUNCH((k_gemm_smallk<TCV, KBV>), grid, dim3(kThreads), 0, st, A, B, (TCV*)C, M, N, K)
  if (c_f32) {
    if (K <= 16) TT_GSK(float, 16); else if (K <= 32) TT_GSK(float, 32); else TT_GSK(float, 64);
  } else {
    if (K <= 16) TT_GSK(double, 16); else if (K <= 32) TT_GSK(double, 32); else TT_GSK(double, 64);
  }
#undef TT_GSK
  return hipGetLastError();
}

int gemm_any_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int64_t s = (K + 255) / 256;                 // at least 256 of k per workgroup
  const int64_t cap = std::max<int64_t>(1, 1024 / tiles);
  if (s > cap) s = cap;
  if (s > 4096) s = 4096;
  return (int)std::max<int64_t>(s, 1);
}

hipError_t launch_gemm_any(const double* A, int64_t sam, int64_t sak, const double* B, int64_t sbk, int64_t sbn,
                           double* C, int64_t M, int64_t N, int64_t K, double* partials, int splits, hipStream_t st) {
  if (M < 1 || N < 1 || K < 1 || splits < 1) return hipErrorInvalidValue;
  const int64_t gx = (M + 63) / 64, gy = (N + 63) / 64;
  if (gy > 65535 || gx > 0x7fffffff || splits > 65535) return hipErrorInvalidValue;
  int64_t kper = (K + splits - 1) / splits;
  kper = (kper + kGaKT - 1) / kGaKT * kGaKT;
  const int z = (int)((K + kper - 1) / kper);   // splits actually used (never an empty one)
  double* dst = (z == 1) ? C : partials;
  if (z > 1 && !partials) return hipErrorInvalidValue;
  TT_LAUNCH(k_gemm_any, dim3((unsigned)gx, (unsigned)gy, (unsigned)z), dim3(kThreads), 0, st, A, sam, sak, B, sbk, sbn,
            dst, M, N, K, kper);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || z == 1) return e;
  return launch_reduce(partials, z, M * N, C, nullptr, st);
}

hipError_t launch_transpose(const double* in, int64_t rows, int64_t cols, double* out, hipStream_t st) {
  if (rows < 1 || cols < 1) return hipErrorInvalidValue;
  const int64_t gx = (rows + 31) / 32, gy = (cols + 31) / 32;
  if (gy > 65535 || gx > 0x7fffffff) return hipErrorInvalidValue;
  TT_LAUNCH(k_transpose, dim3((unsigned)gx, (unsigned)gy), dim3(kThreads), 0, st, in, rows, cols, out);
  return hipGetLastError();
}

static unsigned sample_blocks(int64_t N) {
  int64_t waves = N;
  int64_t blocks = (waves + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

hipError_t launch_sample(int d, const int64_t* dims, const int64_t* ranks,
                         const double* const* cores, const int64_t* idx, int64_t N, double* out,
                         hipStream_t st) {
  TrainDesc D;
  if (!fill_desc(D, d, dims, ranks, cores) || N < 0) return hipErrorInvalidValue;
  if (N == 0) return hipSuccess;
  TT_LAUNCH(k_sample, dim3(sample_blocks(N)), dim3(kThreads), 0, st, D, idx, N, out);
  return hipGetLastError();
}

hipError_t launch_sample_bwd(int d, const int64_t* dims, const int64_t* ranks,
                             const double* const* cores, const double* const* right_cores, const int64_t* idx,
                             int64_t N, const double* gout, double* const* gcores, hipStream_t st) {
  TrainDesc D, DR;
  GradDesc G;
  if (!fill_desc(D, d, dims, ranks, cores)) return hipErrorInvalidValue;
  if (!fill_desc(DR, d, dims, ranks, right_cores ? right_cores : cores)) return hipErrorInvalidValue;
  for (int k = 0; k < d; ++k) G.cores[k] = gcores[k];
  for (int k = 0; k < d; ++k) {
    const int64_t sz = ranks[k] * dims[k] * ranks[k + 1];
    TT_LAUNCH(k_fill_zero, dim3((unsigned)((sz + 255) / 256)), dim3(256), 0, st, gcores[k], sz);
  }
  if (N > 0)
    TT_LAUNCH(k_sample_bwd, dim3(sample_blocks(N)), dim3(kThreads), 0, st, D, DR, idx, N, gout, G);
  return hipGetLastError();
}

}  // namespace ttutv
