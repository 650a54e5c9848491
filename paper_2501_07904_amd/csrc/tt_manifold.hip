// Completion on TT cores (Sec. 4.3, "MRI data completion"): the residual of
// the sampled entries and its energy, the exact line step, the projection of
// core gradients onto the tangent space of the fixed-rank manifold, the cores
// of a tangent vector (or of the point moved along it) and the update of a
// flat vector by a scalar that may live on the device.  Reductions are sums
// of per-workgroup partials in a fixed order, so every result is bitwise
// reproducible.
#include "tt_internal.h"
#include "ttutv.h"

namespace ttutv {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 256;

// fixed-order sum over a 256-thread block: wave sums by shuffles, then the
// four wave sums in wave order
__device__ __forceinline__ double red_block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();   // sh may still be read by a previous sum
  if (lane == 0) sh[w] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

// z = pred - vals; partials[b] = sum of z^2 over block b's share
__global__ __launch_bounds__(kRedThreads) void k_residual(const double* __restrict__ pred,
                                                          const double* __restrict__ vals, int64_t n,
                                                          double* __restrict__ z, double* __restrict__ partials) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads) {
    const double v = pred[i] - vals[i];
    z[i] = v;
    s = fma(v, v, s);
  }
  s = red_block_sum(s, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// partials[2b] = <p, z>, partials[2b + 1] = <p, p> over block b's share
__global__ __launch_bounds__(kRedThreads) void k_line_dots(const double* __restrict__ p,
                                                           const double* __restrict__ z, int64_t n,
                                                           double* __restrict__ partials) {
  __shared__ double sh[4];
  double pz = 0.0, pp = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads) {
    const double a = p[i];
    pz = fma(a, z[i], pz);
    pp = fma(a, a, pp);
  }
  pz = red_block_sum(pz, sh);
  pp = red_block_sum(pp, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = pz;
    partials[2 * blockIdx.x + 1] = pp;
  }
}

// mode 0: out[0] = sum / 2 of nb partials.  mode 1: the line step from nb
// pairs: out = {alpha, <p, z>, <p, p>}, alpha = <p, z> / <p, p> (0 when p = 0)
__global__ __launch_bounds__(kRedThreads) void k_red_finish(const double* __restrict__ partials, int nb, int mode,
                                                            double* __restrict__ out) {
  __shared__ double sh[4];
  if (mode == 0) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) s += partials[b];
    s = red_block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = 0.5 * s;
  } else {
    double pz = 0.0, pp = 0.0;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) {
      pz += partials[2 * b];
      pp += partials[2 * b + 1];
    }
    pz = red_block_sum(pz, sh);
    pp = red_block_sum(pp, sh);
    if (threadIdx.x == 0) {
      out[0] = pp > 0.0 ? pz / pp : 0.0;
      out[1] = pz;
      out[2] = pp;
    }
  }
}

// y += a * s * x, s = *a_dev (or 1)
__global__ __launch_bounds__(kRedThreads) void k_axpy(int64_t n, double a, const double* __restrict__ a_dev,
                                                      const double* __restrict__ x, double* __restrict__ y) {
  const double s = a * (a_dev ? a_dev[0] : 1.0);
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
    y[i] = fma(s, x[i], y[i]);
}

struct TrainPtrs {
  int d;
  int64_t dims[TT_MAX_D];
  int ranks[TT_MAX_D + 1];
  const double* a[TT_MAX_D];   // U (left-orthogonal form)
  const double* b[TT_MAX_D];   // G (projection) or V (tangent train, right-orthogonal form)
  const double* c[TT_MAX_D];   // dC (tangent train)
  double* out[TT_MAX_D];
};

constexpr int kProjTR = 32;   // rows of the left unfoldings staged per round

// Block k: on the left unfoldings ((r0 I) x r1, column-major: the core's own
// layout) dC_k = G_k - U_k (U_k^T G_k) for k < d - 1, dC_{d-1} = G_{d-1}.
// M = U^T G is summed over tiles of 32 rows staged in LDS, every entry of M
// owned by one thread adding the rows in order; then each thread takes rows
// of dC with M in LDS.
__global__ __launch_bounds__(kRedThreads) void k_tangent_project(TrainPtrs P) {
  constexpr int LD = TT_MAX_ELL + 1;
  // two row tiles (U, G) of kProjTR x r1, later M (r1 x r1, stride TT_MAX_ELL)
  __shared__ double sbuf[2 * kProjTR * LD];
  static_assert(2 * kProjTR * LD >= TT_MAX_ELL * TT_MAX_ELL, "M fits in the tile space");
  double* sU = sbuf;
  double* sG = sbuf + kProjTR * LD;
  const int k = blockIdx.x;
  const int r0 = P.ranks[k], r1 = P.ranks[k + 1];
  const int64_t R = (int64_t)r0 * P.dims[k];
  const double* U = P.a[k];
  const double* G = P.b[k];
  double* D = P.out[k];
  const int t = threadIdx.x;
  if (k == P.d - 1) {
    for (int64_t e = t; e < R * r1; e += kRedThreads) D[e] = G[e];
    return;
  }
  constexpr int kPairs = TT_MAX_ELL * TT_MAX_ELL / kRedThreads;   // entries of M per thread
  double acc[kPairs];
#pragma unroll
  for (int j = 0; j < kPairs; ++j) acc[j] = 0.0;
  for (int64_t r00 = 0; r00 < R; r00 += kProjTR) {
    const int nr = (int)(R - r00 < kProjTR ? R - r00 : kProjTR);
    __syncthreads();   // the previous tile has been read
    for (int e = t; e < kProjTR * r1; e += kRedThreads) {
      const int rr = e % kProjTR, col = e / kProjTR;
      sU[rr * LD + col] = rr < nr ? U[r00 + rr + R * col] : 0.0;
      sG[rr * LD + col] = rr < nr ? G[r00 + rr + R * col] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPairs; ++j) {   // entry (a, b): a = lane, b uniform over the wave
      const int pr = t + kRedThreads * j;
      const int a = pr % TT_MAX_ELL, b = pr / TT_MAX_ELL;
      if (a < r1 && b < r1) {
        double s = acc[j];
        for (int rr = 0; rr < kProjTR; ++rr) s = fma(sU[rr * LD + a], sG[rr * LD + b], s);
        acc[j] = s;
      }
    }
  }
  __syncthreads();
  double* sM = sbuf;
#pragma unroll
  for (int j = 0; j < kPairs; ++j) {
    const int pr = t + kRedThreads * j;
    const int a = pr % TT_MAX_ELL, b = pr / TT_MAX_ELL;
    if (a < r1 && b < r1) sM[a + TT_MAX_ELL * b] = acc[j];
  }
  __syncthreads();
  for (int64_t e = t; e < R * r1; e += kRedThreads) {
    const int64_t row = e % R;
    const int b = (int)(e / R);
    double s = 0.0;
    for (int a = 0; a < r1; ++a) s = fma(U[row + R * a], sM[a + TT_MAX_ELL * b], s);
    D[e] = G[e] - s;
  }
}

// Cores of t xi (base = 0) or X + t xi (base = 1), xi = sum_k U_<k dC_k V_>k
// and X = U_1 ... U_d, with ranks (1, 2 r_1, ..., 2 r_{d-1}, 1): first core
// [t dC_1, U_1], interior [[V_k, 0], [t dC_k, U_k]], last [[V_d], [t dC_d (+ U_d)]].
// Block row y = core k; x walks its entries.
__global__ __launch_bounds__(kRedThreads) void k_tangent_train(TrainPtrs P, double t, const double* __restrict__ t_dev,
                                                               int base) {
  const int k = blockIdx.y, d = P.d;
  const double s = t * (t_dev ? t_dev[0] : 1.0);
  const int r0 = P.ranks[k], r1 = P.ranks[k + 1];
  const int64_t I = P.dims[k];
  const int w0 = k == 0 ? 1 : 2 * r0, w1 = k == d - 1 ? 1 : 2 * r1;
  const int64_t n = (int64_t)w0 * I * w1;
  const double* U = P.a[k];
  const double* V = P.b[k];
  const double* C = P.c[k];
  double* W = P.out[k];
  for (int64_t e = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kRedThreads) {
    const int ap = (int)(e % w0);
    const int64_t rest = e / w0;
    const int64_t i = rest % I;
    const int bp = (int)(rest / I);
    double v;
    if (k == 0) {   // r0 = 1
      v = bp < r1 ? s * C[r0 * (i + I * bp)] : U[r0 * (i + I * (bp - r1))];
    } else if (k == d - 1) {   // r1 = 1
      if (ap < r0) v = V[ap + r0 * i];
      else {
        const int64_t o = (ap - r0) + r0 * i;
        v = s * C[o] + (base ? U[o] : 0.0);
      }
    } else if (ap < r0) {
      v = bp < r1 ? V[ap + r0 * (i + I * bp)] : 0.0;
    } else {
      const int a = ap - r0;
      v = bp < r1 ? s * C[a + r0 * (i + I * bp)] : U[a + r0 * (i + I * (bp - r1))];
    }
    W[e] = v;
  }
}

int red_blocks(int64_t n) {
  const int64_t b = (n + kRedThreads - 1) / kRedThreads;
  return (int)(b < 1 ? 1 : (b < kRedBlocks ? b : kRedBlocks));
}

TrainPtrs train_ptrs(int d, const int64_t* dims, const int64_t* ranks, const double* const* a,
                     const double* const* b, const double* const* c, double* const* out) {
  TrainPtrs P;
  P.d = d;
  for (int k = 0; k < d; ++k) {
    P.dims[k] = dims[k];
    P.a[k] = a[k];
    P.b[k] = b[k];
    P.c[k] = c ? c[k] : nullptr;
    P.out[k] = out[k];
  }
  for (int k = 0; k <= d; ++k) P.ranks[k] = (int)ranks[k];
  return P;
}

}  // namespace

size_t reduce_workspace_bytes() { return (size_t)2 * kRedBlocks * sizeof(double); }

hipError_t launch_residual(const double* pred, const double* vals, int64_t n, double* z, double* f, double* work,
                           hipStream_t st) {
  const int nb = red_blocks(n);
  TT_LAUNCH(k_residual, dim3(nb), dim3(kRedThreads), 0, st, pred, vals, n, z, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  TT_LAUNCH(k_red_finish, dim3(1), dim3(kRedThreads), 0, st, work, nb, 0, f);
  return hipGetLastError();
}

hipError_t launch_line_step(const double* p, const double* z, int64_t n, double* out3, double* work,
                            hipStream_t st) {
  const int nb = red_blocks(n);
  TT_LAUNCH(k_line_dots, dim3(nb), dim3(kRedThreads), 0, st, p, z, n, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  TT_LAUNCH(k_red_finish, dim3(1), dim3(kRedThreads), 0, st, work, nb, 1, out3);
  return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, double a, const double* a_dev, const double* x, double* y, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t b = (n + kRedThreads - 1) / kRedThreads;
  TT_LAUNCH(k_axpy, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(kRedThreads), 0, st, n, a, a_dev, x, y);
  return hipGetLastError();
}

hipError_t launch_tangent_project(int d, const int64_t* dims, const int64_t* ranks, const double* const* U,
                                  const double* const* G, double* const* dC, hipStream_t st) {
  TrainPtrs P = train_ptrs(d, dims, ranks, U, G, nullptr, dC);
  TT_LAUNCH(k_tangent_project, dim3(d), dim3(kRedThreads), 0, st, P);
  return hipGetLastError();
}

hipError_t launch_tangent_train(int d, const int64_t* dims, const int64_t* ranks, const double* const* U,
                                const double* const* V, const double* const* dC, double t, const double* t_dev,
                                int base, double* const* W, hipStream_t st) {
  TrainPtrs P = train_ptrs(d, dims, ranks, U, V, dC, W);
  int64_t most = 1;
  for (int k = 0; k < d; ++k) {
    const int64_t w0 = k == 0 ? 1 : 2 * ranks[k], w1 = k == d - 1 ? 1 : 2 * ranks[k + 1];
    const int64_t n = w0 * dims[k] * w1;
    if (n > most) most = n;
  }
  const int64_t b = (most + kRedThreads - 1) / kRedThreads;
  TT_LAUNCH(k_tangent_train, dim3((unsigned)(b < 2048 ? b : 2048), d), dim3(kRedThreads), 0, st, P, t, t_dev, base);
  return hipGetLastError();
}

}  // namespace ttutv
