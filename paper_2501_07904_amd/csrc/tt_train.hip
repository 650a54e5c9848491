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

// ---- sampled entries, one sample per thread --------------------------------
// The forward chain v <- v G_k[:, i_k, :] and the interface products of the
// backward run one sample per thread with the running vector in registers
// (RM >= every rank).  The cores are staged once per workgroup into LDS when
// they fit, each core k as a padded copy with element (a, i, b) at a + P_k (i +
// I_k b), P_k the smallest odd number >= r_{k-1}: the lanes of a wave read the
// same (a, b) of different slices i, and an odd slice stride puts those reads
// on different banks.  Cores that do not fit are read from global memory.
constexpr int kSmpMaxD = 32;
constexpr int kSmpGroups = 256;          // workgroups of the staged kernels (one per CU)
constexpr int kAccThreads = 512;         // gradient accumulation workgroup
constexpr int kAccSB = 128;              // samples staged per accumulation round
constexpr int kLdsMax = 160 * 1024;      // LDS per workgroup on gfx950

struct SmpTrain {
  int d;
  int f32;                           // cores stored as FP32 (else FP64)
  int64_t dims[kSmpMaxD];
  int ranks[kSmpMaxD + 1];
  const void* left[kSmpMaxD];        // cores of the forward chain and of the left products
  const void* right[kSmpMaxD];       // cores of the right products
  int stride[kSmpMaxD];              // a-stride P_k of the padded LDS copies
  int loff[kSmpMaxD];                // LDS offset (doubles) of left core k; -1: global memory
  int roff[kSmpMaxD];                // the same for right core k (== loff when shared)
};

struct LdsAcc {
  const double* base;   // slice i of the padded copy
  int sb;               // stride between b columns
  __device__ __forceinline__ double operator()(int a, int b) const { return base[a + sb * b]; }
};
template <typename TC>
struct GlbAcc {
  const TC* base;       // core + r_{k-1} i
  int64_t sb;           // r_{k-1} I_k
  __device__ __forceinline__ double operator()(int a, int b) const { return (double)base[a + sb * b]; }
};

// nv[b] = sum_{a < ra} v[a] G(a, b) for b < rb; nv[b] = 0 beyond rb
template <int RM, typename ACC>
__device__ __forceinline__ void mv_left(const ACC& G, int ra, int rb, const double* v, double* nv) {
#pragma unroll
  for (int b = 0; b < RM; ++b) {
    double acc = 0.0;
    if (b < rb) {
#pragma unroll
      for (int a = 0; a < RM; ++a)
        if (a < ra) acc = fma(v[a], G(a, b), acc);
    }
    nv[b] = acc;
  }
}
// nr[a] = sum_{b < rb} G(a, b) r[b] for a < ra; nr[a] = 0 beyond ra
template <int RM, typename ACC>
__device__ __forceinline__ void mv_right(const ACC& G, int ra, int rb, const double* r, double* nr) {
#pragma unroll
  for (int a = 0; a < RM; ++a) nr[a] = 0.0;
#pragma unroll
  for (int b = 0; b < RM; ++b) {
    if (b < rb) {
#pragma unroll
      for (int a = 0; a < RM; ++a)
        if (a < ra) nr[a] = fma(G(a, b), r[b], nr[a]);
    }
  }
}

template <int RM>
__device__ __forceinline__ void step_left(const SmpTrain& T, const double* sh, int k, int64_t i, const double* v,
                                          double* nv) {
  const int ra = T.ranks[k], rb = T.ranks[k + 1];
  if (T.loff[k] >= 0)
    mv_left<RM>(LdsAcc{sh + T.loff[k] + (int64_t)T.stride[k] * i, T.stride[k] * (int)T.dims[k]}, ra, rb, v, nv);
  else if (T.f32)
    mv_left<RM>(GlbAcc<float>{(const float*)T.left[k] + ra * i, (int64_t)ra * T.dims[k]}, ra, rb, v, nv);
  else
    mv_left<RM>(GlbAcc<double>{(const double*)T.left[k] + ra * i, (int64_t)ra * T.dims[k]}, ra, rb, v, nv);
}
template <int RM>
__device__ __forceinline__ void step_right(const SmpTrain& T, const double* sh, int k, int64_t i, const double* r,
                                           double* nr) {
  const int ra = T.ranks[k], rb = T.ranks[k + 1];
  if (T.roff[k] >= 0)
    mv_right<RM>(LdsAcc{sh + T.roff[k] + (int64_t)T.stride[k] * i, T.stride[k] * (int)T.dims[k]}, ra, rb, r, nr);
  else if (T.f32)
    mv_right<RM>(GlbAcc<float>{(const float*)T.right[k] + ra * i, (int64_t)ra * T.dims[k]}, ra, rb, r, nr);
  else
    mv_right<RM>(GlbAcc<double>{(const double*)T.right[k] + ra * i, (int64_t)ra * T.dims[k]}, ra, rb, r, nr);
}

// copy the cores marked for LDS into their padded layout
template <int NTH>
__device__ __forceinline__ void stage_cores(const SmpTrain& T, double* sh) {
  for (int k = 0; k < T.d; ++k) {
    for (int side = 0; side < 2; ++side) {
      const int off = side ? T.roff[k] : T.loff[k];
      if (off < 0 || (side == 1 && T.roff[k] == T.loff[k])) continue;
      const void* src = side ? T.right[k] : T.left[k];
      const int ra = T.ranks[k], rb = T.ranks[k + 1];
      const int64_t I = T.dims[k];
      const int64_t n = (int64_t)ra * I * rb;
      for (int64_t e = threadIdx.x; e < n; e += NTH) {
        const int a = (int)(e % ra);
        const int64_t rest = e / ra;
        const int64_t i = rest % I, b = rest / I;
        const double x = T.f32 ? (double)((const float*)src)[e] : ((const double*)src)[e];
        sh[off + a + (int64_t)T.stride[k] * (i + I * b)] = x;
      }
    }
  }
}

// out[s] = the train's entry at row s of idx
template <int RM, int NTH>
__global__ __launch_bounds__(NTH) void k_sample_t(SmpTrain T, const int64_t* __restrict__ idx, int64_t N,
                                                  double* __restrict__ out) {
  extern __shared__ double sh[];
  stage_cores<NTH>(T, sh);
  __syncthreads();
  const int d = T.d;
  for (int64_t s = (int64_t)blockIdx.x * NTH + threadIdx.x; s < N; s += (int64_t)gridDim.x * NTH) {
    const int64_t* ix = idx + s * d;
    double v[RM], nv[RM];
#pragma unroll
    for (int a = 0; a < RM; ++a) v[a] = a == 0 ? 1.0 : 0.0;
    for (int k = 0; k < d; ++k) {
      step_left<RM>(T, sh, k, ix[k], v, nv);
#pragma unroll
      for (int a = 0; a < RM; ++a) v[a] = nv[a];
    }
    out[s] = v[0];
  }
}

// Interface products of samples s0 .. s0+nb-1 (one per thread): for every
// core k, L_k[s] = gout[s] * G_1[i_1] ... G_{k-1}[i_{k-1}] (r_{k-1} entries,
// left cores) and R_k[s] = G_{k+1}[i_{k+1}] ... G_d[i_d] (r_k entries, right
// cores), stored entry-major at ws + lo[k] and ws + ro[k]: entry a of sample
// q at a * nb + q, so the 64 samples of a wave write 512 contiguous bytes.
struct IfaceOut {
  int64_t lo[kSmpMaxD], ro[kSmpMaxD];
};
template <int RM, int NTH>
__global__ __launch_bounds__(NTH) void k_sample_iface(SmpTrain T, const int64_t* __restrict__ idx, int64_t s0,
                                                      int64_t nb, const double* __restrict__ gout,
                                                      double* __restrict__ ws, IfaceOut O) {
  extern __shared__ double sh[];
  stage_cores<NTH>(T, sh);
  __syncthreads();
  const int d = T.d;
  for (int64_t q = (int64_t)blockIdx.x * NTH + threadIdx.x; q < nb; q += (int64_t)gridDim.x * NTH) {
    const int64_t s = s0 + q;
    const int64_t* ix = idx + s * d;
    const double w = gout[s];
    double v[RM], nv[RM];
#pragma unroll
    for (int a = 0; a < RM; ++a) v[a] = a == 0 ? 1.0 : 0.0;
    for (int k = 0; k < d; ++k) {
      const int ra = T.ranks[k];
      double* L = ws + O.lo[k] + q;
#pragma unroll
      for (int a = 0; a < RM; ++a)
        if (a < ra) L[(int64_t)a * nb] = w * v[a];
      if (k + 1 < d) {
        step_left<RM>(T, sh, k, ix[k], v, nv);
#pragma unroll
        for (int a = 0; a < RM; ++a) v[a] = nv[a];
      }
    }
#pragma unroll
    for (int a = 0; a < RM; ++a) v[a] = a == 0 ? 1.0 : 0.0;
    for (int k = d - 1; k >= 0; --k) {
      const int rb = T.ranks[k + 1];
      double* R = ws + O.ro[k] + q;
#pragma unroll
      for (int b = 0; b < RM; ++b)
        if (b < rb) R[(int64_t)b * nb] = v[b];
      if (k > 0) {
        step_right<RM>(T, sh, k, ix[k], v, nv);
#pragma unroll
        for (int a = 0; a < RM; ++a) v[a] = nv[a];
      }
    }
  }
}

// Gradient of core k over samples s0 .. s0+nb-1 from their interface
// products, on the FP64 matrix cores: the gradient is I_k slices of r_{k-1} x
// r_k, each sum over the samples with i_k = i of L_s R_s^T, cut into 16 x 16
// tiles.  Workgroup w takes a contiguous share of the samples and stages 128
// of them at a time in LDS (their L, R and i_k); wave v owns tiles tau0 + v,
// tau0 + v + 8, ... (at most eight, the accumulators held in registers for
// the whole launch).  For a tile of slice i the wave finds the staged samples
// with i_k = i by a ballot and feeds them four at a time, in sample order, as
// the k dimension of v_mfma_f64_16x16x4 (operand A: L_s[a], lane (g, l) ->
// sample g, a = l; operand B: R_s[b]).  Every tile has one owner and the
// order of its products is fixed, so the partial sums do not depend on
// timing; a workgroup starts from its partial of the previous sample block
// (partials + w * total) unless `first`, and the partials are summed over
// workgroups in a fixed order afterwards.
struct AccDesc {
  int d;
  int64_t dims[kSmpMaxD];
  int ranks[kSmpMaxD + 1];
  int64_t coff[kSmpMaxD + 1];
  IfaceOut O;
};

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kAccTilesPerWave = 8;

template <int NTH>
__global__ __launch_bounds__(NTH) void k_grad_mfma(AccDesc A, const int64_t* __restrict__ idx, int64_t s0, int64_t nb,
                                                   const double* __restrict__ ws, double* __restrict__ partials,
                                                   int64_t total, int first, int k, int tau0, int tau1, int lda) {
  constexpr int NW = NTH / 64;
  extern __shared__ double sh[];
  double* stl = sh;                               // [kAccSB][lda]: L_s
  double* str = stl + kAccSB * lda;               // [kAccSB][lda]: R_s
  int* sti = (int*)(str + kAccSB * lda);          // [kAccSB]: i_k of the staged samples
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int d = A.d;
  const int ra = A.ranks[k], rb = A.ranks[k + 1];
  const int I = (int)A.dims[k];
  const int tpa = (ra + 15) / 16, tps = tpa * ((rb + 15) / 16);   // tiles per slice
  const int64_t coff = A.coff[k];
  double* mine = partials + (int64_t)blockIdx.x * total;
  d4 acc[kAccTilesPerWave];
#pragma unroll
  for (int j = 0; j < kAccTilesPerWave; ++j) {
    acc[j] = d4{0.0, 0.0, 0.0, 0.0};
    const int tau = tau0 + wv + NW * j;
    if (!first && tau < tau1) {
      const int i = tau / tps, ta = (tau % tps) % tpa, tb = (tau % tps) / tpa;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * ta + g + 4 * v, b = 16 * tb + li;
        if (a < ra && b < rb) acc[j][v] = mine[coff + a + (int64_t)ra * (i + (int64_t)I * b)];
      }
    }
  }
  const int64_t per = (nb + gridDim.x - 1) / gridDim.x;
  const int64_t q_beg = min(nb, (int64_t)blockIdx.x * per), q_end = min(nb, q_beg + per);
  const double* L = ws + A.O.lo[k];
  const double* Rv = ws + A.O.ro[k];
  // the next round's staged values are loaded into registers while the
  // current round runs on the matrix cores, then stored to LDS behind a barrier
  constexpr int NPF = kAccSB * 32 / NTH;   // values per thread, ranks <= 32
  double pl[NPF], pr[NPF];
  int pi = 0;
  auto fetch = [&](int64_t q0) {
#pragma unroll
    for (int u = 0; u < NPF; ++u) {   // entry e / kAccSB of staged sample e % kAccSB
      const int e = t + NTH * u;
      const int q = e % kAccSB, a = e / kAccSB;
      const bool in = q0 + q < q_end;
      pl[u] = (a < ra && in) ? L[(int64_t)a * nb + q0 + q] : 0.0;
      pr[u] = (a < rb && in) ? Rv[(int64_t)a * nb + q0 + q] : 0.0;
    }
    pi = (t < kAccSB && q0 + t < q_end) ? (int)idx[(s0 + q0 + t) * d + k] : -1;
  };
  if (q_beg < q_end) fetch(q_beg);
  for (int64_t q0 = q_beg; q0 < q_end; q0 += kAccSB) {
    __syncthreads();   // the previous round's reads of the staging area are done
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int e = t + NTH * u;
      const int q = e % kAccSB, a = e / kAccSB;
      if (a < ra) stl[q * lda + a] = pl[u];
      if (a < rb) str[q * lda + a] = pr[u];
    }
    if (t < kAccSB) sti[t] = pi;
    __syncthreads();
    if (q0 + kAccSB < q_end) fetch(q0 + kAccSB);
    const int key0 = sti[lane], key1 = sti[64 + lane];   // -1 past the last staged sample
#pragma unroll
    for (int j = 0; j < kAccTilesPerWave; ++j) {
      const int tau = tau0 + wv + NW * j;
      if (tau >= tau1) continue;   // uniform
      const int i = tau / tps, ta = (tau % tps) % tpa, tb = (tau % tps) / tpa;
      uint64_t m0 = __ballot(key0 == i), m1 = __ballot(key1 == i);
      const int a = 16 * ta + li, b = 16 * tb + li;
      while (m0 | m1) {   // uniform: four samples of slice i per step, in sample order
        int sg = -1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          int sq = -1;
          if (m0) {
            sq = __ffsll((unsigned long long)m0) - 1;
            m0 &= m0 - 1;
          } else if (m1) {
            sq = 64 + __ffsll((unsigned long long)m1) - 1;
            m1 &= m1 - 1;
          }
          if (g == u) sg = sq;
        }
        const double lv = (sg >= 0 && a < ra) ? stl[sg * lda + a] : 0.0;
        const double rv = (sg >= 0 && b < rb) ? str[sg * lda + b] : 0.0;
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv, rv, acc[j], 0, 0, 0);
      }
    }
  }
  // result register v of lane (g, l): row a = 16 ta + g + 4 v, column b = 16 tb + l
#pragma unroll
  for (int j = 0; j < kAccTilesPerWave; ++j) {
    const int tau = tau0 + wv + NW * j;
    if (tau >= tau1) continue;
    const int i = tau / tps, ta = (tau % tps) % tpa, tb = (tau % tps) / tpa;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * ta + g + 4 * v, b = 16 * tb + li;
      if (a < ra && b < rb) mine[coff + a + (int64_t)ra * (i + (int64_t)I * b)] = acc[j][v];
    }
  }
}

// gcores[k][e - coff[k]] = sum over workgroups of the partials, fixed order
struct GradOut {
  void* cores[kSmpMaxD];
  int64_t coff[kSmpMaxD + 1];
  int d;
  int f32;
};
// A block sums 16 consecutive entries: thread (g, j) adds partials
// g*per .. g*per+per-1 of entry j in order, then the 16 group sums are added
// in group order (a fixed order; 16 groups keep enough loads in flight).
constexpr int kRedEntries = 16, kRedGroups = kThreads / kRedEntries;
__global__ __launch_bounds__(kThreads) void k_grad_reduce(const double* __restrict__ partials, int nparts,
                                                          int64_t total, GradOut G) {
  __shared__ double sh[kRedGroups][kRedEntries];
  const int j = threadIdx.x % kRedEntries, g = threadIdx.x / kRedEntries;
  const int64_t e = (int64_t)blockIdx.x * kRedEntries + j;
  const int per = (nparts + kRedGroups - 1) / kRedGroups;
  double s = 0.0;
  if (e < total) {
    const int w1 = min(nparts, (g + 1) * per);
    for (int w = g * per; w < w1; ++w) s += partials[(int64_t)w * total + e];
  }
  sh[g][j] = s;
  __syncthreads();
  if (g != 0 || e >= total) return;
  s = sh[0][j];
  for (int q = 1; q < kRedGroups; ++q) s += sh[q][j];
  int k = 0;
  while (k + 1 < G.d && e >= G.coff[k + 1]) ++k;
  const int64_t o = e - G.coff[k];
  if (G.f32) ((float*)G.cores[k])[o] = (float)s;
  else ((double*)G.cores[k])[o] = s;
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
  // a workgroup's k loop is a chain of dependent load / barrier / FMA rounds
  // (kGaKT of k each), so on the narrow outputs of a train's chain rule
  // (M or N a rank) its length, not the arithmetic, sets the time: one round
  // per workgroup where the partials (s M N doubles, summed afterwards) stay
  // within 2^21 doubles and the workgroups within 4096
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int64_t s = (K + kGaKT - 1) / kGaKT;
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(4096 / tiles, ((int64_t)1 << 21) / (M * N)));
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

// ---- host side of the one-sample-per-thread kernels -------------------------
namespace {

constexpr int64_t kBwdBlock = (int64_t)1 << 20;   // samples per interface block of the backward

struct SmpPlan {
  SmpTrain T;
  int rm;                // register vector length: 8, 16 or 32
  size_t lds;            // bytes of staged cores
  int64_t total;         // gradient entries of the concatenated cores
  int64_t coff[kSmpMaxD + 1];
};

int smp_rm(int d, const int64_t* ranks) {
  int64_t r = 1;
  for (int k = 0; k <= d; ++k) r = std::max(r, ranks[k]);
  return r <= 8 ? 8 : r <= 16 ? 16 : r <= 32 ? 32 : 0;
}

// Cores into LDS while the padded copies fit in `budget` bytes: the left set
// first, then the right set when it is a different train.
bool smp_plan(int d, const int64_t* dims, const int64_t* ranks, const void* const* left, const void* const* right,
              int f32, size_t budget, SmpPlan& P) {
  if (d < 2 || d > kSmpMaxD) return false;
  P.rm = smp_rm(d, ranks);
  if (!P.rm) return false;
  SmpTrain& T = P.T;
  T.d = d;
  T.f32 = f32;
  P.coff[0] = 0;
  for (int k = 0; k <= d; ++k) T.ranks[k] = (int)ranks[k];
  for (int k = 0; k < d; ++k) {
    T.dims[k] = dims[k];
    T.left[k] = left[k];
    T.right[k] = right ? right[k] : left[k];
    T.stride[k] = (int)(ranks[k] | 1);
    P.coff[k + 1] = P.coff[k] + ranks[k] * dims[k] * ranks[k + 1];
  }
  P.total = P.coff[d];
  if (P.total >= ((int64_t)1 << 31)) return false;   // 32-bit entry offsets in the accumulation
  int64_t need_l = 0;
  for (int k = 0; k < d; ++k) need_l += (int64_t)T.stride[k] * dims[k] * ranks[k + 1];
  const bool same = !right || right == left;
  int64_t used = 0;
  const bool lds_l = need_l * 8 <= (int64_t)budget;
  for (int k = 0; k < d; ++k) {
    T.loff[k] = lds_l ? (int)used : -1;
    if (lds_l) used += (int64_t)T.stride[k] * dims[k] * ranks[k + 1];
  }
  const bool lds_r = !same && (used + need_l) * 8 <= (int64_t)budget;
  for (int k = 0; k < d; ++k) {
    if (same) { T.roff[k] = T.loff[k]; continue; }
    T.roff[k] = lds_r ? (int)used : -1;
    if (lds_r) used += (int64_t)T.stride[k] * dims[k] * ranks[k + 1];
  }
  P.lds = (size_t)used * 8;
  return true;
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

unsigned smp_grid(int64_t n, int nth, size_t lds) {
  int64_t g = (n + nth - 1) / nth;
  const int64_t cap = lds > 0 ? kSmpGroups : 2048;   // staged cores: one workgroup per CU
  if (g > cap) g = cap;
  return (unsigned)std::max<int64_t>(g, 1);
}

template <int RM, int NTH>
hipError_t run_sample(const SmpPlan& P, const int64_t* idx, int64_t N, double* out, hipStream_t st) {
  hipError_t e = allow_lds(k_sample_t<RM, NTH>, P.lds);
  if (e != hipSuccess) return e;
  TT_LAUNCH((k_sample_t<RM, NTH>), dim3(smp_grid(N, NTH, P.lds)), dim3(NTH), P.lds, st, P.T, idx, N, out);
  return hipGetLastError();
}

template <int RM, int NTH>
hipError_t run_iface(const SmpPlan& P, const int64_t* idx, int64_t s0, int64_t nb, const double* gout, double* ws,
                     const IfaceOut& O, hipStream_t st) {
  hipError_t e = allow_lds(k_sample_iface<RM, NTH>, P.lds);
  if (e != hipSuccess) return e;
  TT_LAUNCH((k_sample_iface<RM, NTH>), dim3(smp_grid(nb, NTH, P.lds)), dim3(NTH), P.lds, st, P.T, idx, s0, nb,
            gout, ws, O);
  return hipGetLastError();
}

// LDS of the accumulation: two staged rows of lda = rm + 1 doubles per sample
// (rows 2 banks apart for the four samples a matrix-core step reads) and the
// slice indices
size_t acc_lds_bytes(int rm) { return (size_t)2 * kAccSB * (rm + 1) * 8 + kAccSB * 4 + 64; }

// iface block (doubles) and partials (doubles) of the backward
void bwd_sizes(int d, const int64_t* ranks, int64_t N, int64_t total, int64_t* iface, int64_t* parts) {
  int64_t per = 0;
  for (int k = 0; k < d; ++k) per += ranks[k] + ranks[k + 1];
  *iface = std::min<int64_t>(std::max<int64_t>(N, 1), kBwdBlock) * per;
  *parts = (int64_t)kSmpGroups * total;
}

}  // namespace

int sample_rm(int d, const int64_t* ranks) { return smp_rm(d, ranks); }

hipError_t launch_sample2(int d, const int64_t* dims, const int64_t* ranks, const void* const* cores, int f32,
                          const int64_t* idx, int64_t N, double* out, hipStream_t st) {
  SmpPlan P;
  if (!smp_plan(d, dims, ranks, cores, nullptr, f32, kLdsMax, P) || N < 0) return hipErrorInvalidValue;
  if (N == 0) return hipSuccess;
  switch (P.rm) {
    case 8: return run_sample<8, 1024>(P, idx, N, out, st);
    case 16: return run_sample<16, 1024>(P, idx, N, out, st);
    default: return run_sample<32, 512>(P, idx, N, out, st);
  }
}

size_t sample_bwd2_workspace(int d, const int64_t* dims, const int64_t* ranks, int64_t N) {
  int64_t total = 0;
  for (int k = 0; k < d; ++k) total += ranks[k] * dims[k] * ranks[k + 1];
  int64_t iface, parts;
  bwd_sizes(d, ranks, N, total, &iface, &parts);
  return (size_t)(iface + parts) * 8 + 256;
}

hipError_t launch_sample_bwd2(int d, const int64_t* dims, const int64_t* ranks, const void* const* left,
                              const void* const* right, int f32, const int64_t* idx, int64_t N, const double* gout,
                              void* const* gcores, void* work, size_t work_bytes, hipStream_t st) {
  SmpPlan P;
  if (!smp_plan(d, dims, ranks, left, right, f32, kLdsMax, P) || N < 0) return hipErrorInvalidValue;
  if (work_bytes < sample_bwd2_workspace(d, dims, ranks, N)) return hipErrorInvalidValue;
  int64_t iface, parts;
  bwd_sizes(d, ranks, N, P.total, &iface, &parts);
  double* ws = (double*)(((uintptr_t)work + 255) & ~(uintptr_t)255);
  double* partials = ws + iface;
  GradOut G;
  G.d = d;
  G.f32 = f32;
  for (int k = 0; k < d; ++k) G.cores[k] = gcores[k];
  for (int k = 0; k <= d; ++k) G.coff[k] = P.coff[k];
  if (N == 0) {
    // no samples: every partial is zero
    TT_LAUNCH(k_fill_zero, dim3((unsigned)((parts + 255) / 256)), dim3(256), 0, st, partials, parts);
  } else {
    const int64_t cap = std::min<int64_t>(N, kBwdBlock);
    IfaceOut O;
    int64_t off = 0;
    for (int k = 0; k < d; ++k) {
      O.lo[k] = off;
      off += cap * ranks[k];
      O.ro[k] = off;
      off += cap * ranks[k + 1];
    }
    AccDesc A;
    A.d = d;
    A.O = O;
    for (int k = 0; k < d; ++k) A.dims[k] = dims[k];
    for (int k = 0; k <= d; ++k) {
      A.ranks[k] = (int)ranks[k];
      A.coff[k] = P.coff[k];
    }
    const size_t acc_lds = acc_lds_bytes(P.rm);
    hipError_t e = allow_lds(k_grad_mfma<kAccThreads>, acc_lds);
    if (e != hipSuccess) return e;
    constexpr int tiles_per_launch = (kAccThreads / 64) * kAccTilesPerWave;
    for (int64_t s0 = 0; s0 < N; s0 += cap) {
      const int64_t nb = std::min(cap, N - s0);
      switch (P.rm) {
        case 8: e = run_iface<8, 1024>(P, idx, s0, nb, gout, ws, O, st); break;
        case 16: e = run_iface<16, 1024>(P, idx, s0, nb, gout, ws, O, st); break;
        default: e = run_iface<32, 512>(P, idx, s0, nb, gout, ws, O, st); break;
      }
      if (e != hipSuccess) return e;
      for (int k = 0; k < d; ++k) {
        const int tiles = (int)(dims[k] * ((ranks[k] + 15) / 16) * ((ranks[k + 1] + 15) / 16));
        for (int tau0 = 0; tau0 < tiles; tau0 += tiles_per_launch) {
          const int tau1 = std::min(tiles, tau0 + tiles_per_launch);
          TT_LAUNCH(k_grad_mfma<kAccThreads>, dim3(kSmpGroups), dim3(kAccThreads), acc_lds, st, A, idx, s0, nb, ws,
                    partials, P.total, s0 == 0 ? 1 : 0, k, tau0, tau1, P.rm + 1);
          e = hipGetLastError();
          if (e != hipSuccess) return e;
        }
      }
    }
  }
  TT_LAUNCH(k_grad_reduce, dim3((unsigned)((P.total + kRedEntries - 1) / kRedEntries)), dim3(kThreads), 0, st,
            partials, kSmpGroups, P.total, G);
  return hipGetLastError();
}

}  // namespace ttutv
