// Single-workgroup FP64 factorisations of the small side of a step: the
// Gaussian test matrix, Householder orthonormalisation of n x ell blocks, the
// symmetric eigen-decomposition of the ell x ell Rayleigh-Ritz matrix by
// cyclic Jacobi, the rank decision and the core fold.
#include "tt_internal.h"

namespace ttutv {

namespace {

constexpr int kThreads = 256;
constexpr int kLd = kCMax + 1;   // padded leading dimension of LDS matrices

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kThreads / 64; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// --------------------------------------------------------------------------
// SplitMix64: the t-th output from state `seed` is the xor-shift-multiply
// finaliser applied to seed + t * golden-ratio increment.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t t) {
  uint64_t z = seed + t * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Gaussian entry of the test matrix for mode index i, carried-rank index
// beta and column j of the step producing core `label`: counter
// c = label<<48 | j<<32 | beta<<16 | i, uniforms from outputs 2c+1 and 2c+2,
// Box-Muller sqrt(-2 ln u1) cos(2 pi u2).
__device__ __forceinline__ double sketch_entry(uint64_t seed, int label, int i, int beta, int j) {
  const uint64_t c = ((uint64_t)label << 48) | ((uint64_t)j << 32) | ((uint64_t)beta << 16) | (uint64_t)i;
  const uint64_t x1 = splitmix64_at(seed, 2 * c + 1);
  const uint64_t x2 = splitmix64_at(seed, 2 * c + 2);
  const double u1 = ((double)(x1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(2.0 * 3.141592653589793 * u2);
}

__device__ __forceinline__ double sketch_row_entry(const SolveArgs& a, int row, int j) {
  int i, beta;
  if (a.mode_fastest) { i = row % a.n_mode; beta = row / a.n_mode; }
  else { beta = row % a.n_rank; i = row / a.n_rank; }
  return sketch_entry(a.seed, a.label, i, beta, j);
}

__global__ void k_gen_sketch(double* G, SolveArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)a.n * a.ell) return;
  G[e] = sketch_row_entry(a, (int)(e % a.n), (int)(e / a.n));
}

// --------------------------------------------------------------------------
// Householder QR of X (n x c, column-major, leading dim ldx), c <= 64: X is
// overwritten by the reflectors and Q (n x c) receives the explicit
// orthonormal factor H_0 H_1 ... H_{c-1} [I; 0].  A zero column gives an
// identity reflector, so Q stays orthonormal for rank-deficient X.
__device__ void householder_q(double* X, int64_t ldx, double* Q, int64_t ldq, int n, int c,
                              double* tau, double* sh) {
  const int t = threadIdx.x;
  for (int k = 0; k < c; ++k) {
    double part = 0.0;
    for (int i = k + 1 + t; i < n; i += kThreads) {
      const double x = X[i + k * ldx];
      part = fma(x, x, part);
    }
    const double sig = block_sum(part, sh);
    if (t == 0) {
      const double alpha = X[k + k * ldx];
      double tk = 0.0, scale = 0.0;
      if (sig > 0.0) {
        const double mu = sqrt(fma(alpha, alpha, sig));
        const double beta = alpha <= 0.0 ? mu : -mu;
        tk = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
        X[k + k * ldx] = beta;
      }
      tau[k] = tk;
      sh[8] = scale;
    }
    __syncthreads();
    const double tk = tau[k];
    const double scale = sh[8];
    if (tk != 0.0) {
      for (int i = k + 1 + t; i < n; i += kThreads) X[i + k * ldx] *= scale;
    }
    __syncthreads();
    const int ncol = c - k - 1;
    if (ncol > 0 && tk != 0.0) {
      int tpj = 64;
      while (tpj * ncol > kThreads && tpj > 1) tpj >>= 1;
      const int col = t / tpj, lane = t % tpj;
      const bool on = col < ncol;
      const int j = k + 1 + col;
      double dot = 0.0;
      if (on) {
        if (lane == 0) dot = X[k + j * ldx];
        for (int i = k + 1 + lane; i < n; i += tpj) dot = fma(X[i + k * ldx], X[i + j * ldx], dot);
      }
      for (int o = tpj >> 1; o > 0; o >>= 1) dot += __shfl_xor(dot, o, 64);
      if (on) {
        const double f = tk * dot;
        if (lane == 0) X[k + j * ldx] -= f;
        for (int i = k + 1 + lane; i < n; i += tpj) X[i + j * ldx] = fma(-f, X[i + k * ldx], X[i + j * ldx]);
      }
    }
    __syncthreads();
  }
  for (int64_t e = t; e < (int64_t)n * c; e += kThreads) {
    const int i = (int)(e % n), j = (int)(e / n);
    Q[i + j * ldq] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = c - 1; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;
    const int ncol = c - k;
    int tpj = 64;
    while (tpj * ncol > kThreads && tpj > 1) tpj >>= 1;
    const int col = t / tpj, lane = t % tpj;
    const bool on = col < ncol;
    const int j = k + col;
    double dot = 0.0;
    if (on) {
      if (lane == 0) dot = Q[k + j * ldq];
      for (int i = k + 1 + lane; i < n; i += tpj) dot = fma(X[i + k * ldx], Q[i + j * ldq], dot);
    }
    for (int o = tpj >> 1; o > 0; o >>= 1) dot += __shfl_xor(dot, o, 64);
    if (on) {
      const double f = tk * dot;
      if (lane == 0) Q[k + j * ldq] -= f;
      for (int i = k + 1 + lane; i < n; i += tpj) Q[i + j * ldq] = fma(-f, X[i + k * ldx], Q[i + j * ldq]);
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// Symmetric eigen-decomposition of K (L x L in LDS, ld kLd) by cyclic Jacobi
// with the round-robin parallel ordering (L/2 disjoint rotations per round).
// On return lam[0..L) holds the eigenvalues in descending order and perm[a]
// the column of Z (L x L, ld kLd) holding the eigenvector of lam[a].
__device__ void jacobi_eig(double* K, double* Z, int L, double* lam, int* perm, double* rot,
                           int* rp, double* sh, int* flag) {
  const int t = threadIdx.x;
  const int Le = L + (L & 1);
  for (int e = t; e < L * L; e += kThreads) {
    const int i = e % L, j = e / L;
    Z[i + j * kLd] = (i == j) ? 1.0 : 0.0;
  }
  double dmax_part = 0.0;
  for (int i = t; i < L; i += kThreads) dmax_part = fmax(dmax_part, fabs(K[i + i * kLd]));
  // block max via shuffles + LDS
  for (int o = 32; o > 0; o >>= 1) dmax_part = fmax(dmax_part, __shfl_xor(dmax_part, o, 64));
  if ((t & 63) == 0) sh[t >> 6] = dmax_part;
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < kThreads / 64; ++i) dmax = fmax(dmax, sh[i]);
  __syncthreads();
  const double abs_floor = 1e-300 + 1e-18 * dmax;
  for (int sweep = 0; sweep < 40 && Le >= 2; ++sweep) {
    if (t == 0) *flag = 0;
    __syncthreads();
    for (int round = 0; round < Le - 1; ++round) {
      if (t < Le / 2) {
        const int p = t;
        int a, b;
        if (p == 0) { a = 0; b = 1 + (round % (Le - 1)); }
        else { a = 1 + ((p + round) % (Le - 1)); b = 1 + ((Le - 1 - p + round) % (Le - 1)); }
        if (a > b) { const int s = a; a = b; b = s; }
        double cs = 1.0, sn = 0.0;
        if (b < L) {
          const double app = K[a + a * kLd], aqq = K[b + b * kLd], apq = K[a + b * kLd];
          if (fabs(apq) > abs_floor && fabs(apq) > 1e-15 * sqrt(fabs(app) * fabs(aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            cs = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * cs;
            *flag = 1;
          }
        }
        rot[p] = cs;
        rot[32 + p] = sn;
        rp[p] = a;
        rp[32 + p] = b;
      }
      __syncthreads();
      // K <- J^T K: rows a, b
      for (int e = t; e < (Le / 2) * L; e += kThreads) {
        const int p = e / L, j = e % L;
        const double cs = rot[p], sn = rot[32 + p];
        if (sn == 0.0) continue;
        const int a = rp[p], b = rp[32 + p];
        const double ka = K[a + j * kLd], kb = K[b + j * kLd];
        K[a + j * kLd] = cs * ka - sn * kb;
        K[b + j * kLd] = sn * ka + cs * kb;
      }
      __syncthreads();
      // K <- K J and Z <- Z J: columns a, b
      for (int e = t; e < (Le / 2) * L; e += kThreads) {
        const int p = e / L, i = e % L;
        const double cs = rot[p], sn = rot[32 + p];
        if (sn == 0.0) continue;
        const int a = rp[p], b = rp[32 + p];
        const double ka = K[i + a * kLd], kb = K[i + b * kLd];
        K[i + a * kLd] = cs * ka - sn * kb;
        K[i + b * kLd] = sn * ka + cs * kb;
        const double za = Z[i + a * kLd], zb = Z[i + b * kLd];
        Z[i + a * kLd] = cs * za - sn * zb;
        Z[i + b * kLd] = sn * za + cs * zb;
      }
      __syncthreads();
    }
    const int any = *flag;
    __syncthreads();
    if (!any) break;
  }
  // descending order, ties by index
  if (t < L) {
    const double v = K[t + t * kLd];
    int rank = 0;
    for (int j = 0; j < L; ++j) {
      const double w = K[j + j * kLd];
      rank += (w > v) || (w == v && j < t);
    }
    perm[rank] = t;
  }
  __syncthreads();
  if (t < L) lam[t] = K[perm[t] + perm[t] * kLd];
  __syncthreads();
}

// Rank decision (fixed r, or the smallest r with ||C||^2 - sum_{i<=r} s_i^2 <= eps_k^2).
__device__ void decide_rank(const SolveArgs& a, const double* lam, int ell, double normC2,
                            double normA2, int* out_r, int* out_sat, double* out_kept) {
  int r, sat;
  if (a.r_fixed > 0) {
    r = min(a.r_fixed, ell);
    sat = 1;
  } else {
    const double eps2 = a.eps_factor2 * normA2;
    double kept = 0.0;
    r = ell;
    sat = 0;
    for (int i = 0; i < ell; ++i) {
      kept += fmax(lam[i], 0.0);
      if (normC2 - kept <= eps2) { r = i + 1; sat = 1; break; }
    }
    const int cap = a.max_rank > 0 ? a.max_rank : kCMax;
    if (r > cap) { r = cap; sat = 0; }
  }
  if (r < 1) r = 1;
  double kept = 0.0;
  for (int i = 0; i < r; ++i) kept += fmax(lam[i], 0.0);
  *out_r = r;
  *out_sat = sat;
  *out_kept = kept;
}

// Column signs: largest-magnitude entry of every column of V (n x r) positive,
// lowest row on ties; one wave per column.
__device__ void canonical_signs(const double* V, int64_t ldv, int n, int r, double* sg) {
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int a = w; a < r; a += kThreads / 64) {
    double best = -1.0, val = 0.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < n; i += 64) {
      const double x = V[i + a * ldv];
      const double ax = fabs(x);
      if (ax > best) { best = ax; bi = i; val = x; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      const double ov = __shfl_xor(val, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; val = ov; }
    }
    if (lane == 0) sg[a] = (val < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
}

// --------------------------------------------------------------------------
// Gram mode: H = A^T A is n x n with n <= 64.  X spans H^(q+1) G (or is the
// identity when ell = n); Rayleigh-Ritz on X gives the rank-revealing
// factorisation; the core side V1 = X Z_r goes to the core and to V1.
__global__ __launch_bounds__(kThreads) void k_gram_solve(const double* __restrict__ H, SolveArgs a) {
  __shared__ double sH[kCMax * kLd];
  __shared__ double sX[kCMax * kLd];
  __shared__ double sQ[kCMax * kLd];
  __shared__ double sK[kCMax * kLd];
  __shared__ double lam[kCMax], tau[kCMax], rot[64], sg[kCMax], sh[16];
  __shared__ int perm[kCMax], rp[64], flag, sr, ssat;
  __shared__ double skept, snormC2;
  const int t = threadIdx.x;
  const int n = a.n;
  const int ell = min(a.ell, n);
  for (int e = t; e < n * n; e += kThreads) sH[(e % n) + (e / n) * kLd] = H[e];
  __syncthreads();
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += sH[i + i * kLd];
    const double nc2 = a.normC2_src ? *a.normC2_src : tr;
    snormC2 = nc2;
    if (a.first) *a.normA2 = nc2;
  }
  if (ell >= n) {
    for (int e = t; e < n * n; e += kThreads) sX[(e % n) + (e / n) * kLd] = ((e % n) == (e / n)) ? 1.0 : 0.0;
  } else {
    for (int e = t; e < n * ell; e += kThreads) sX[(e % n) + (e / n) * kLd] = sketch_row_entry(a, e % n, e / n);
  }
  __syncthreads();
  const int L = ell >= n ? n : ell;
  if (ell < n) {
    for (int it = 0; it <= a.q; ++it) {
      for (int e = t; e < n * L; e += kThreads) {
        const int i = e % n, j = e / n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = fma(sH[i + k * kLd], sX[k + j * kLd], s);
        sQ[i + j * kLd] = s;
      }
      __syncthreads();
      householder_q(sQ, kLd, sX, kLd, n, L, tau, sh);
    }
  }
  // K = X^T H X
  for (int e = t; e < n * L; e += kThreads) {
    const int i = e % n, j = e / n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s = fma(sH[i + k * kLd], sX[k + j * kLd], s);
    sQ[i + j * kLd] = s;
  }
  __syncthreads();
  for (int e = t; e < L * L; e += kThreads) {
    const int i = e % L, j = e / L;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s = fma(sX[k + i * kLd], sQ[k + j * kLd], s);
    sK[i + j * kLd] = s;
  }
  __syncthreads();
  // symmetrise against rounding
  for (int e = t; e < L * L; e += kThreads) {
    const int i = e % L, j = e / L;
    if (i < j) {
      const double v = 0.5 * (sK[i + j * kLd] + sK[j + i * kLd]);
      sK[i + j * kLd] = v;
      sK[j + i * kLd] = v;
    }
  }
  __syncthreads();
  double* sZ = sH;  // H is no longer needed
  jacobi_eig(sK, sZ, L, lam, perm, rot, rp, sh, &flag);
  if (t == 0) {
    int r, sat;
    double kept;
    decide_rank(a, lam, L, snormC2, *a.normA2, &r, &sat, &kept);
    sr = r; ssat = sat; skept = kept;
  }
  __syncthreads();
  const int r = sr;
  // V1 = X Z_r (into sQ)
  for (int e = t; e < n * r; e += kThreads) {
    const int i = e % n, c = e / n;
    const int pc = perm[c];
    double s = 0.0;
    for (int k = 0; k < L; ++k) s = fma(sX[i + k * kLd], sZ[k + pc * kLd], s);
    sQ[i + c * kLd] = s;
  }
  __syncthreads();
  canonical_signs(sQ, kLd, n, r, sg);
  for (int e = t; e < n * r; e += kThreads) {
    const int i = e % n, c = e / n;
    const double v = sQ[i + c * kLd] * sg[c];
    a.V1[i + (int64_t)n * c] = v;
    if (a.core) {
      if (a.core_layout == 0) a.core[i + (int64_t)n * c] = v;
      else a.core[c + (int64_t)r * i] = v;
    }
  }
  if (t == 0) {
    StepRec* rec = a.rec;
    rec->normC2 = snormC2;
    rec->kept2 = skept;
    rec->r = r;
    rec->sat = ssat;
    rec->ell = L;
    rec->resid2 = -1.0;
  }
  for (int i = t; i < kCMax; i += kThreads) a.rec->lam[i] = (i < L) ? lam[i] : 0.0;
}

// --------------------------------------------------------------------------
// X = orth(M) for n x c blocks; LDS-resident when it fits, else in place in
// global memory (M is overwritten by the reflectors).
constexpr int kOrthLdsDoubles = 8192;

__global__ __launch_bounds__(kThreads) void k_orth(double* M, double* X, int n, int c) {
  __shared__ double buf[2 * kOrthLdsDoubles];
  __shared__ double tau[kCMax], sh[16];
  const int t = threadIdx.x;
  if ((int64_t)n * c <= kOrthLdsDoubles) {
    double* sM = buf;
    double* sX = buf + kOrthLdsDoubles;
    for (int e = t; e < n * c; e += kThreads) sM[e] = M[e];
    __syncthreads();
    householder_q(sM, n, sX, n, n, c, tau, sh);
    for (int e = t; e < n * c; e += kThreads) X[e] = sX[e];
  } else {
    householder_q(M, n, X, n, n, c, tau, sh);
  }
}

// --------------------------------------------------------------------------
// Rayleigh-Ritz on span(X) from K = Y^T Y (Y = A X): eigen-decomposition
// K = Z diag(lam) Z^T, rank decision, V1 = X Z_r (core side), W = Z_r so that
// the carry A V1 equals Y W.
__global__ __launch_bounds__(kThreads) void k_rr_solve(const double* __restrict__ K,
                                                       const double* __restrict__ X, SolveArgs a) {
  __shared__ double sK[kCMax * kLd];
  __shared__ double sZ[kCMax * kLd];
  __shared__ double lam[kCMax], rot[64], sg[kCMax], sh[16];
  __shared__ int perm[kCMax], rp[64], flag, sr, ssat;
  __shared__ double skept, snormC2;
  const int t = threadIdx.x;
  const int n = a.n;
  const int L = a.ell;
  for (int e = t; e < L * L; e += kThreads) {
    const int i = e % L, j = e / L;
    sK[i + j * kLd] = 0.5 * (K[i + (int64_t)L * j] + K[j + (int64_t)L * i]);
  }
  if (t == 0) snormC2 = *a.normC2_src;
  __syncthreads();
  jacobi_eig(sK, sZ, L, lam, perm, rot, rp, sh, &flag);
  if (t == 0) {
    int r, sat;
    double kept;
    decide_rank(a, lam, L, snormC2, *a.normA2, &r, &sat, &kept);
    sr = r; ssat = sat; skept = kept;
  }
  __syncthreads();
  const int r = sr;
  for (int64_t e = t; e < (int64_t)n * r; e += kThreads) {
    const int i = (int)(e % n), c = (int)(e / n);
    const int pc = perm[c];
    double s = 0.0;
    for (int k = 0; k < L; ++k) s = fma(X[i + (int64_t)n * k], sZ[k + pc * kLd], s);
    a.V1[e] = s;
  }
  __threadfence_block();
  __syncthreads();
  canonical_signs(a.V1, n, n, r, sg);
  for (int64_t e = t; e < (int64_t)n * r; e += kThreads) {
    const int i = (int)(e % n), c = (int)(e / n);
    const double v = a.V1[e] * sg[c];
    a.V1[e] = v;
    if (a.core) {
      if (a.core_layout == 0) a.core[i + (int64_t)n * c] = v;
      else a.core[c + (int64_t)r * i] = v;
    }
  }
  for (int e = t; e < L * r; e += kThreads) {
    const int k = e % L, c = e / L;
    a.W[k + (int64_t)L * c] = sZ[k + perm[c] * kLd] * sg[c];
  }
  if (t == 0) {
    StepRec* rec = a.rec;
    rec->normC2 = snormC2;
    rec->kept2 = skept;
    rec->r = r;
    rec->sat = ssat;
    rec->ell = L;
    rec->resid2 = -1.0;
  }
  for (int i = t; i < kCMax; i += kThreads) a.rec->lam[i] = (i < L) ? lam[i] : 0.0;
}

}  // namespace

hipError_t launch_gram_solve(const double* H, const SolveArgs& a, hipStream_t st) {
  if (a.n < 1 || a.n > kGramMax || a.ell < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gram_solve, dim3(1), dim3(kThreads), 0, st, H, a);
  return hipGetLastError();
}

hipError_t launch_gen_sketch(double* G, const SolveArgs& a, hipStream_t st) {
  const int64_t total = (int64_t)a.n * a.ell;
  if (total < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gen_sketch, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, G, a);
  return hipGetLastError();
}

hipError_t launch_orth(double* M, double* X, int n, int c, hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || c > n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_orth, dim3(1), dim3(kThreads), 0, st, M, X, n, c);
  return hipGetLastError();
}

hipError_t launch_rr_solve(const double* K, const double* X, const SolveArgs& a, hipStream_t st) {
  if (a.n < 1 || a.ell < 1 || a.ell > kCMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rr_solve, dim3(1), dim3(kThreads), 0, st, K, X, a);
  return hipGetLastError();
}

}  // namespace ttutv
