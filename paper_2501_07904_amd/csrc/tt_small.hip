// Single-workgroup FP64 factorisations of the small side of a step: the
// Gaussian test matrix, Householder orthonormalisation of n x ell blocks, the
// symmetric eigen-decomposition of the ell x ell Rayleigh-Ritz matrix by
// cyclic Jacobi, the rank decision and the core fold.
#include "tt_internal.h"

namespace ttutv {

namespace {

constexpr int kThreads = 1024;   // single-workgroup solvers: 16 waves
constexpr int kLd = kCMax + 1;   // padded leading dimension of LDS matrices

// Cross-lane sums without LDS round trips: DPP moves inside rows of 16
// lanes, then v_readlane across the rows of a wave.  Every lane of a group
// ends with the bit-identical sum (each pairing adds the same two operands).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]: pairs
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]: quads
  v += dpp_mov<0x141>(v);   // row_half_mirror: lane i with 7-i, eights
  v += dpp_mov<0x140>(v);   // row_mirror: lane i with 15-i, rows of 16
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of tpj lanes, tpj in {16, 32, 64}; the lanes of a
// summed row must all be active.
__device__ __forceinline__ double group_sum(double v, int tpj) {
  v = row16_sum(v);
  if (tpj == 16) return v;
  const double r0 = readlane_d(v, 0), r1 = readlane_d(v, 16);
  const double r2 = readlane_d(v, 32), r3 = readlane_d(v, 48);
  if (tpj == 32) return (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
  return (r0 + r1) + (r2 + r3);
}

// sqrt(x) and 1/sqrt(x) for x > 0: the hardware reciprocal-square-root
// estimate refined by two coupled (Goldschmidt) steps carrying sqrt(x) and
// 1/(2 sqrt(x)) together (each step squares the relative error).
__device__ __forceinline__ void sqrt_rsq(double x, double* sq, double* rs) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, hf = 0.5 * y;
  double r = fma(-g, hf, 0.5);
  g = fma(g, r, g);
  hf = fma(hf, r, hf);
  r = fma(-g, hf, 0.5);
  *sq = fma(g, r, g);
  *rs = 2.0 * fma(hf, r, hf);
}

// Two group sums at once, their DPP steps interleaved (one reduction's latency).
__device__ __forceinline__ void group_sum2(double* a, double* b, int tpj) {
  double u = *a, v = *b;
  u += dpp_mov<0xB1>(u);
  v += dpp_mov<0xB1>(v);
  u += dpp_mov<0x4E>(u);
  v += dpp_mov<0x4E>(v);
  u += dpp_mov<0x141>(u);
  v += dpp_mov<0x141>(v);
  u += dpp_mov<0x140>(u);
  v += dpp_mov<0x140>(v);
  if (tpj == 16) { *a = u; *b = v; return; }
  const double u0 = readlane_d(u, 0), u1 = readlane_d(u, 16), u2 = readlane_d(u, 32), u3 = readlane_d(u, 48);
  const double v0 = readlane_d(v, 0), v1 = readlane_d(v, 16), v2 = readlane_d(v, 32), v3 = readlane_d(v, 48);
  if (tpj == 32) {
    const bool hi = threadIdx.x & 32;
    *a = hi ? u2 + u3 : u0 + u1;
    *b = hi ? v2 + v3 : v0 + v1;
    return;
  }
  *a = (u0 + u1) + (u2 + u3);
  *b = (v0 + v1) + (v2 + v3);
}

// x . v over a thread's R rows: four partial sums (R is a multiple of 4).
template <int R>
__device__ __forceinline__ double dot_rows(const double* x, const double* v) {
  double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < R; ++r) d[r & 3] = fma(v[r], x[r], d[r & 3]);
  return (d[0] + d[1]) + (d[2] + d[3]);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = group_sum(v, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kThreads / 64; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// ||C||^2 of a step: the previous carry's partial sums of squares reduced by
// the whole block (strided per thread, then block_sum: a fixed order), or the
// stored value.  Every thread gets the result; thread 0 records the sum.
__device__ __forceinline__ double step_norm2(const SolveArgs& a, double* sh) {
  if (!a.nc_parts) return *a.normC2_src;
  double v = 0.0;
  for (int e = threadIdx.x; e < a.nc_n; e += kThreads) v += a.nc_parts[e];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) *a.nc_out = s;
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
  const int row = (int)(e / a.ell), j = (int)(e % a.ell);
  // k-major: G[row * ell + j]; ell >= n means the exact step, G = I
  G[e] = (a.ell >= a.n) ? (row == j ? 1.0 : 0.0) : sketch_row_entry(a, row, j);
}

// --------------------------------------------------------------------------
// Householder QR of X (n x c, c <= 64) with the explicit orthonormal factor
// Q = H_0 ... H_{c-1} [I; 0] formed backwards (as LAPACK's dorg2r does); a
// column already zero below the diagonal gives the identity reflector, so Q
// stays orthonormal for rank-deficient X.  Register-resident, for n <= R * tpj:
// thread group g (tpj threads, tpj = kThreads / c rounded up to a power of
// two) owns column g and keeps its rows i = lane + tpj*r (r < R) in registers.  Column k's Householder vector
// is published by its group through a double-buffered LDS vector, so both the
// factorisation and the backward formation of Q take one barrier per column.
// Input X(i, j) at X[i*xi + j*xj]; output Q(i, j) at Q[i*qi + j*qj] (may alias X).
__host__ __device__ __forceinline__ int reg_group_width(int c) {
  int cp = 1;
  while (cp < c) cp <<= 1;
  const int tpj = kThreads / cp;
  return tpj < 64 ? tpj : 64;
}

// Rout (optional): the c x c triangular factor R(i, j) at Rout[i*ri + j*rj],
// zero below the diagonal, with M = Q R.
template <int R, int TPJ>
__device__ __forceinline__ void householder_reg(const double* X, int64_t xi, int64_t xj, double* Q, int64_t qi,
                                                int64_t qj, int n, int c, double* vbuf, double* Rout = nullptr,
                                                int64_t ri = 0, int64_t rj = 0, double* vall = nullptr) {
  // rows are padded to NP = R * TPJ with zeros, so the loops below need no row
  // guards; TPJ (= reg_group_width(c)) is a compile-time constant so that the
  // LDS offsets of a thread's rows are immediates.  Step k of the
  // factorisation first applies H_{k-1} to the columns g >= k, then group k
  // forms reflector k from its freshly updated column: one barrier per step.
  const int t = threadIdx.x;
  constexpr int NP = R * TPJ;
  const int g = t / TPJ, lane = t % TPJ;
  const bool own = g < c;
  double x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + TPJ * r;
    x[r] = (own && i < n) ? X[i * xi + g * xj] : 0.0;
  }
  double* taus = vbuf + 2 * NP;
  double my_tau = 0.0, my_diag = 0.0;
  // ---- factorisation
  for (int k = 0; k < c; ++k) {
    if (k > 0 && own && g >= k) {
      const double* v = vbuf + ((k - 1) & 1) * NP + lane;
      const double tk = taus[k - 1];
      double vr[R];
#pragma unroll
      for (int r = 0; r < R; ++r) vr[r] = v[TPJ * r];
      const double f = tk * group_sum(dot_rows<R>(x, vr), TPJ);
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = fma(-f, vr[r], x[r]);
    }
    if (g == k) {
      double sg4[4] = {0.0, 0.0, 0.0, 0.0}, alpha = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + TPJ * r;
        sg4[r & 3] = fma(i > k ? x[r] : 0.0, x[r], sg4[r & 3]);
        alpha = (i == k) ? x[r] : alpha;
      }
      double sig = (sg4[0] + sg4[1]) + (sg4[2] + sg4[3]);
      group_sum2(&sig, &alpha, TPJ);   // one lane holds row k, the others add zero to alpha
      double tk = 0.0, sc = 0.0;
      my_diag = alpha;   // R(k, k): alpha when column k is already zero below row k, else beta
      if (sig > 0.0) {
        // mu = sqrt(alpha^2 + sig) and 1/mu together; beta = -sign(alpha) mu,
        // tau = (beta - alpha) / beta, and the scale 1 / (alpha - beta), where
        // |alpha - beta| = |alpha| + mu lies in [mu, 2 mu]: a reciprocal
        // estimate refined by two Newton steps
        double mu, rmu;
        sqrt_rsq(fma(alpha, alpha, sig), &mu, &rmu);
        const bool neg = alpha <= 0.0;
        const double beta = neg ? mu : -mu;
        tk = (beta - alpha) * (neg ? rmu : -rmu);
        const double dn = alpha - beta;
        double q = __builtin_amdgcn_rcp(dn);
        q = fma(q, fma(-dn, q, 1.0), q);
        sc = fma(q, fma(-dn, q, 1.0), q);
        my_diag = beta;
      }
      my_tau = tk;
      double* v = vbuf + (k & 1) * NP + lane;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + TPJ * r;
        const double vi = (i < k) ? 0.0 : (i == k ? 1.0 : sc * x[r]);
        v[TPJ * r] = vi;
        x[r] = (i > k) ? vi : x[r];   // keep the scaled reflector below the diagonal
      }
      if (lane == 0) taus[k] = tk;
    }
    __syncthreads();
  }
  if (Rout && own) {
    // column g: rows above the diagonal hold R, row g keeps alpha (R(g, g) is my_diag)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + TPJ * r;
      if (i < c) Rout[i * ri + g * rj] = (i < g) ? x[r] : (i == g ? my_diag : 0.0);
    }
  }
  // ---- Q = H_0 ... H_{c-1} [I; 0]; column g is H_0 ... H_g e_g, since
  // H_k e_g = e_g for k > g
  if (vall) {
    // all reflectors are known: publish them together (vall holds NP x c),
    // then every group forms its own column, H_g e_g followed by H_{g-1}, ...,
    // H_0, with no further barrier (the same operations in the same order as
    // the step-wise loop below)
    if (own) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + TPJ * r;
        vall[g * NP + i] = (i < g) ? 0.0 : (i == g ? 1.0 : x[r]);
      }
    }
    __syncthreads();
    if (own) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + TPJ * r;
        x[r] = (i < g) ? 0.0 : (i == g ? 1.0 - my_tau : -my_tau * x[r]);
      }
      for (int k = g - 1; k >= 0; --k) {
        const double* v = vall + k * NP + lane;
        const double tk = taus[k];
        double vr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) vr[r] = v[TPJ * r];
        const double f = tk * group_sum(dot_rows<R>(x, vr), TPJ);
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = fma(-f, vr[r], x[r]);
      }
    }
  }
  // step-wise: group k publishes v_k, the groups g > k apply H_k to their
  // columns, group k forms H_k e_k
  for (int k = c - 1; k >= 0 && !vall; --k) {
    if (g == k) {
      double* v = vbuf + (k & 1) * NP + lane;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + TPJ * r;
        v[TPJ * r] = (i < k) ? 0.0 : (i == k ? 1.0 : x[r]);
      }
      if (lane == 0) taus[k] = my_tau;
    }
    __syncthreads();
    if (own && g > k) {
      const double* v = vbuf + (k & 1) * NP + lane;
      const double tk = taus[k];
      double vr[R];
#pragma unroll
      for (int r = 0; r < R; ++r) vr[r] = v[TPJ * r];
      const double f = tk * group_sum(dot_rows<R>(x, vr), TPJ);
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = fma(-f, vr[r], x[r]);
    } else if (g == k) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + TPJ * r;
        x[r] = (i < k) ? 0.0 : (i == k ? 1.0 - my_tau : -my_tau * x[r]);
      }
    }
  }
  __syncthreads();   // every read of X (and of vbuf) is done before Q may overwrite them
  if (own) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + TPJ * r;
      if (i < n) Q[i * qi + g * qj] = x[r];
    }
  }
  __syncthreads();
}


// Rows per thread the register path needs for an n x c block (0: too large).
__device__ __host__ __forceinline__ int reg_rows(int n, int c) {
  int cp = 1;
  while (cp < c) cp <<= 1;
  int tpj = kThreads / cp;
  if (tpj > 64) tpj = 64;
  const int R = (n + tpj - 1) / tpj;
  return R <= 4 ? 4 : R <= 8 ? 8 : R <= 16 ? 16 : 0;   // R <= 16 keeps 1024 threads within 128 VGPRs
}

// --------------------------------------------------------------------------
// Symmetric eigen-decomposition of K (L x L in LDS, ld kLd) by cyclic Jacobi
// with the round-robin parallel ordering: each round rotates L/2 disjoint
// pairs, and K <- J^T K J is applied as independent 2 x 2 block updates.
// Pairs whose off-diagonal entry is below the rounding floor are skipped; the
// iteration stops before a sweep that would rotate nothing, or once sweeps no
// longer reduce the off-diagonal mass.
// On return lam[0..L) holds the eigenvalues in descending order and perm[a]
// the column of Z (L x L, ld kLd) holding the eigenvector of lam[a].
//
// Pair p of round r (0 <= r < m = Le - 1, Le = L rounded up to even) holds
// the indices x = 0, y = 1 + r for p = 0 and x = 1 + (p + r) mod m,
// y = 1 + (m - p + r) mod m otherwise.  From one round to the next an index
// moves by at most one pair position: the x member of pair p + 1 becomes the
// x member of pair p, the y member of pair p - 1 the y member of pair p, and
// the ends turn around (pair 0's y comes from pair 1's x, pair 1's y from
// pair 0's y, the last pair's x from its own y).
__device__ __forceinline__ void pair_labels(int p, int r, int m, int* x, int* y) {
  // r < m and p <= m / 2, so each sum is below 2m: one conditional subtraction
  int u = p + r;
  if (u >= m) u -= m;
  int v = m - p + r;
  if (v >= m) v -= m;
  *x = p == 0 ? 0 : 1 + u;
  *y = p == 0 ? 1 + r : 1 + v;
}

// Position (pair, member) in the previous round of member s of pair p.
__device__ __forceinline__ void pair_source(int p, int s, int h, int* po, int* so) {
  if (h == 1) { *po = p; *so = s; return; }
  if (p == 0) { *po = s; *so = 0; return; }
  if (s == 0) {
    if (p < h - 1) { *po = p + 1; *so = 0; }
    else { *po = h - 1; *so = 1; }
  } else {
    if (p == 1) { *po = 0; *so = 1; }
    else { *po = p - 1; *so = 1; }
  }
}

// Rotation (cs, sn) of a pair with diagonal entries app, aqq and coupling
// apq, zeroing apq; the identity when apq is below the rounding floor.
// With d = aqq - app and w = 2 apq scaled by the same power of two to
// max(|d|, |w|) in [1/2, 1) (exact; the angle is scale invariant) and
// h = sqrt(d^2 + w^2), D = |d| + h:  tan(theta) = sign(d) w / D (the root of
// magnitude at most 1), so cs = D / sqrt(D^2 + w^2) and
// sn = sign(d) w / sqrt(D^2 + w^2), with no division.  Both square roots come
// from the hardware reciprocal-square-root estimate refined by two coupled
// (Goldschmidt) steps that carry sqrt(x) and 1/(2 sqrt(x)) together; cs and
// sn share the same 1/sqrt, so the rotation is orthogonal to working
// accuracy.  Every thread that evaluates a pair does so from the same
// operands with the same operations, so all copies agree bitwise.

__device__ __forceinline__ void jacobi_rot(double app, double aqq, double apq, double abs_floor, double* cs,
                                           double* sn) {
  const bool on = fabs(apq) > abs_floor && apq * apq > 1e-30 * fabs(app * aqq);
  const double dd = aqq - app, tw = 2.0 * apq;
  int ex;
  (void)frexp(fmax(fabs(dd), fabs(tw)), &ex);
  const double d1 = ldexp(dd, -ex), w1 = ldexp(tw, -ex);
  const double w2 = w1 * w1;
  double hq, unused;
  sqrt_rsq(fma(d1, d1, w2), &hq, &unused);
  const double den = fabs(d1) + hq;   // in [1/2, 1 + sqrt(2))
  double rn, y;
  sqrt_rsq(fma(den, den, w2), &rn, &y);
  (void)rn;
  (void)unused;
  *cs = on ? den * y : 1.0;
  *sn = on ? (d1 >= 0.0 ? w1 : -w1) * y : 0.0;
}

// K is L x L in LDS (ld kLd); K2 is scratch of the same size.  During the
// iteration K is held by pair position rather than by index: entry (i, j),
// with i member si of pair Pi and j member sj of pair Pj in the current round,
// sits in plane si + 2 sj at Pi + h Pj (four planes of h x h, h = Le / 2).
// The thread of block (P, Q) writes its four entries at P + h Q and, the next
// round, reads them from where the pair movement above put them: offsets
// fixed for the whole solve, and the lanes of a wave touch nearly consecutive
// words of each plane (an index-addressed layout has 4- to 8-way LDS bank
// conflicts on the same accesses).  The rounds alternate between K2 and K.
// Z stays index-addressed; the thread of block (P, Q) rotates rows 2P, 2P + 1
// of the columns of pair Q.
template <int NT>
__device__ __forceinline__ int jacobi_eig(double* K, double* K2, double* Z, int L, double* lam, int* perm,
                                          double* sh, int* flag) {
  // K and Z are padded to Le = L rounded up to even with a zero row and column;
  // the pair holding the padding index then always gets the identity rotation
  const int t = threadIdx.x;
  const int Le = L + (L & 1);
  const int h = Le / 2, m = Le - 1, hh = h * h;
  for (int e = t; e < Le * Le; e += NT) {
    const int i = e % Le, j = e / Le;
    Z[i + j * kLd] = (i == j && i < L) ? 1.0 : 0.0;
  }
  double dpart = 0.0;
  for (int i = t; i < L; i += NT) dpart = fmax(dpart, fabs(K[i + i * kLd]));
  for (int o = 32; o > 0; o >>= 1) dpart = fmax(dpart, __shfl_xor(dpart, o, 64));
  if ((t & 63) == 0) sh[t >> 6] = dpart;
  // perm serves as the index -> position table (2 pair + member) of the layout
  // written by the last round of a sweep (round m - 1), which is also the
  // layout the first round reads
  if (t < h) {
    int x, y;
    pair_labels(t, m - 1 > 0 ? m - 1 : 0, m, &x, &y);
    perm[x] = 2 * t;
    perm[y] = 2 * t + 1;
  }
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < NT / 64; ++i) dmax = fmax(dmax, sh[i]);
  // rotations stop at the rounding floor: below 1e-15 of the largest diagonal
  // entry and of the geometric mean of the pair's diagonal entries (looser
  // floors were measured to cost eigenvector accuracy of small, well
  // separated eigenvalues)
  const double abs_floor = 1e-300 + 1e-15 * dmax;
  for (int e = t; e < Le * Le; e += NT) {
    const int i = e % Le, j = e / Le;
    const int pi = perm[i], pj = perm[j];
    K2[((pi & 1) + 2 * (pj & 1)) * hh + (pi >> 1) + h * (pj >> 1)] = (i < L && j < L) ? K[i + j * kLd] : 0.0;
  }
  __syncthreads();
  double* Kc = K2;
  double* Kn = K;
  int sweeps = 0;
  static_assert(NT >= (kCMax / 2) * (kCMax / 2), "one 2 x 2 block per thread");
  // a round is two phases: thread p < h evaluates the rotation of pair p
  // (lam holds the h rotations meanwhile) while every block thread loads its
  // block and Z entries; after a barrier the block threads apply the
  // rotations of their two pairs
  const bool blk = t < hh;            // this thread's block (P, Q), fixed for the whole solve
  const int P = t % h, Q = blk ? t / h : 0;
  double* rot = lam;
  int Pa, sa, Pb, sb, Qa, ta, Qb, tb;
  pair_source(P, 0, h, &Pa, &sa);
  pair_source(P, 1, h, &Pb, &sb);
  pair_source(Q, 0, h, &Qa, &ta);
  pair_source(Q, 1, h, &Qb, &tb);
  const int o_pa = 3 * sa * hh + Pa * (1 + h), o_pb = 3 * sb * hh + Pb * (1 + h);
  const int o_pab = (sa + 2 * sb) * hh + Pa + h * Pb;
  const int o_aa = (sa + 2 * ta) * hh + Pa + h * Qa, o_ab = (sa + 2 * tb) * hh + Pa + h * Qb;
  const int o_ba = (sb + 2 * ta) * hh + Pb + h * Qa, o_bb = (sb + 2 * tb) * hh + Pb + h * Qb;
  const int own = P + h * Q;
  double prev_off2 = HUGE_VAL;
  for (int sweep = 0; sweep < 30 && L >= 2; ++sweep) {
    // converged when no pair would be rotated: exactly the sweep that would
    // follow applies no rotation, so it is not run
    if (t == 0) *flag = 0;
    __syncthreads();
    double off = 0.0;
    for (int e = t; e < 4 * hh; e += NT) {
      const int pl = e / hh, idx = e - pl * hh;
      const int Pi = idx % h, Pj = idx / h;
      if (Pi == Pj && (pl == 0 || pl == 3)) continue;   // a diagonal entry
      const double apq = Kc[e];
      off = fma(apq, apq, off);
      const double di = Kc[3 * (pl & 1) * hh + Pi * (1 + h)], dj = Kc[3 * (pl >> 1) * hh + Pj * (1 + h)];
      if (fabs(apq) > abs_floor && apq * apq > 1e-30 * fabs(di * dj)) *flag = 1;
    }
    for (int o = 32; o > 0; o >>= 1) off += __shfl_xor(off, o, 64);
    if ((t & 63) == 0) sh[t >> 6] = off;
    __syncthreads();
    const int any = *flag;
    double off2 = 0.0;
    for (int i = 0; i < NT / 64; ++i) off2 += sh[i];
    __syncthreads();
    // also stop once the off-diagonal mass no longer falls (by 4x per sweep
    // after the first four): the entries left above the floor are then
    // rounding noise of the large ones that further rotations only move around
    if (!any || (sweep >= 4 && off2 > 0.25 * prev_off2)) break;
    prev_off2 = off2;
    sweeps = sweep + 1;
    for (int round = 0; round < m; ++round) {
      // phase 1: the rotations (threads t < h hold pair t as their row pair)
      if (t < h) {
        const double pa = Kc[o_pa], pb = Kc[o_pb], pab = Kc[o_pab];
        double cP, sP;
        jacobi_rot(pa, pb, pab, abs_floor, &cP, &sP);
        rot[2 * t] = cP;
        rot[2 * t + 1] = sP;
      }
      double kaa = 0.0, kab = 0.0, kba = 0.0, kbb = 0.0, z0a = 0.0, z0b = 0.0, z1a = 0.0, z1b = 0.0;
      double* z0 = Z;
      double* z1 = Z;
      if (blk) {
        kaa = Kc[o_aa]; kab = Kc[o_ab]; kba = Kc[o_ba]; kbb = Kc[o_bb];
        int xQ, yQ;
        pair_labels(Q, round, m, &xQ, &yQ);
        z0 = Z + 2 * P + xQ * kLd;
        z1 = Z + 2 * P + yQ * kLd;
        z0a = z0[0]; z0b = z0[1]; z1a = z1[0]; z1b = z1[1];
      }
      __syncthreads();
      // phase 2: the block update
      if (blk) {
        const double cP = rot[2 * P], sP = rot[2 * P + 1], cQ = rot[2 * Q], sQ = rot[2 * Q + 1];
        const double raa = cQ * kaa - sQ * kab, rab = sQ * kaa + cQ * kab;
        const double rba = cQ * kba - sQ * kbb, rbb = sQ * kba + cQ * kbb;
        Kn[own] = cP * raa - sP * rba;              // (x_P, x_Q)
        Kn[hh + own] = sP * raa + cP * rba;         // (y_P, x_Q)
        Kn[2 * hh + own] = cP * rab - sP * rbb;     // (x_P, y_Q)
        Kn[3 * hh + own] = sP * rab + cP * rbb;     // (y_P, y_Q)
        // Z <- Z J on rows 2P, 2P + 1 and the columns of pair Q
        z0[0] = cQ * z0a - sQ * z1a;
        z0[1] = cQ * z0b - sQ * z1b;
        z1[0] = sQ * z0a + cQ * z1a;
        z1[1] = sQ * z0b + cQ * z1b;
      }
      __syncthreads();
      double* tmp = Kc; Kc = Kn; Kn = tmp;
    }
  }
  // descending order, ties by index; the diagonal is read through the
  // position table before perm is overwritten
  double v = 0.0;
  if (t < L) {
    const int pi = perm[t];
    v = Kc[3 * (pi & 1) * hh + (pi >> 1) * (1 + h)];
  }
  __syncthreads();
  if (t < L) lam[t] = v;
  __syncthreads();
  int rank = 0;
  if (t < L) {
    for (int j = 0; j < L; ++j) {
      const double w = lam[j];
      rank += (w > v) || (w == v && j < t);
    }
  }
  __syncthreads();
  if (t < L) {
    perm[rank] = t;
    lam[rank] = v;
  }
  __syncthreads();
  return sweeps;
}

// Rank decision (fixed r, or the smallest r with ||C||^2 - sum_{i<=r} s_i^2 <= eps_k^2).
__device__ __forceinline__ void decide_rank(const SolveArgs& a, const double* lam, int ell, double normC2,
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
template <int NT>
__device__ __forceinline__ void canonical_signs(const double* V, int64_t si, int64_t sa, int n, int r, double* sg) {
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int a = w; a < r; a += NT / 64) {
    double best = -1.0, val = 0.0;
    int bi = 0x7fffffff;
    // rows in increasing order per lane, four loads in flight
    for (int i0 = lane; i0 < n; i0 += 256) {
      double xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u;
        xv[u] = i < n ? V[i * si + a * sa] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u;
        const double ax = fabs(xv[u]);
        if (i < n && ax > best) { best = ax; bi = i; val = xv[u]; }
      }
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
  __shared__ double sB0[kCMax * kLd];
  __shared__ double sB1[kCMax * kLd];
  __shared__ double sK[kCMax * kLd];
  __shared__ double lam[kCMax], tau[kCMax], scal[kCMax], sg[kCMax], sh[32];
  __shared__ double vbuf[2 * 64 * 4 + kCMax];   // register Householder with R = 4, tpj <= 64
  __shared__ int perm[kCMax], flag, sr, ssat;
  __shared__ double skept, snormC2;
  const int t = threadIdx.x;
  const int n = a.n;
  const int L = min(a.ell, n);
  for (int e = t; e < n * n; e += kThreads) sH[(e % n) + (e / n) * kLd] = H[e];
  double* X = sB0;   // current basis (n x L)
  double* T = sB1;   // H X
  if (L >= n) {
    for (int e = t; e < n * n; e += kThreads) X[(e % n) + (e / n) * kLd] = ((e % n) == (e / n)) ? 1.0 : 0.0;
  } else {
    for (int e = t; e < n * L; e += kThreads) X[(e % n) + (e / n) * kLd] = sketch_row_entry(a, e % n, e / n);
  }
  __syncthreads();
  const double prev_nc2 = (a.nc_parts || a.normC2_src) ? step_norm2(a, sh) : 0.0;
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += sH[i + i * kLd];
    const double nc2 = (a.nc_parts || a.normC2_src) ? prev_nc2 : tr;
    snormC2 = nc2;
    if (a.first) *a.normA2 = nc2;
  }
  if (L < n) {
    // X spans H^(q+1) G: multiply, orthonormalise in place, swap
    for (int it = 0; it <= a.q; ++it) {
      for (int e = t; e < n * L; e += kThreads) {
        const int i = e % n, j = e / n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = fma(sH[i + k * kLd], X[k + j * kLd], s);
        T[i + j * kLd] = s;
      }
      __syncthreads();
      // n <= 64: at most 4 rows per thread; sK (free until K is formed) holds
      // the reflectors for the barrier-free formation of Q
      static_assert(kCMax * kLd >= 4 * kThreads, "sK holds 4 * kThreads doubles");
      // rows per thread: just enough for n (every padded row costs LDS reads
      // of the reflectors in each step)
      const int tpj = reg_group_width(L);
      const int rn = (n + tpj - 1) / tpj;
#define TT_GHH(RV, TV) householder_reg<RV, TV>(T, 1, kLd, T, 1, kLd, n, L, vbuf, nullptr, 0, 0, sK)
      if (tpj == 16) {
        if (rn <= 1) TT_GHH(1, 16); else if (rn <= 2) TT_GHH(2, 16); else TT_GHH(4, 16);
      } else if (tpj == 32) {
        if (rn <= 1) TT_GHH(1, 32); else TT_GHH(2, 32);
      } else {
        TT_GHH(1, 64);
      }
#undef TT_GHH
      double* tmp = X; X = T; T = tmp;
    }
  }
  // K = X^T H X
  for (int e = t; e < n * L; e += kThreads) {
    const int i = e % n, j = e / n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s = fma(sH[i + k * kLd], X[k + j * kLd], s);
    T[i + j * kLd] = s;
  }
  __syncthreads();
  for (int e = t; e < L * L; e += kThreads) {
    const int i = e % L, j = e / L;
    if (i > j) continue;
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < n; ++k) {
      s1 = fma(X[k + i * kLd], T[k + j * kLd], s1);
      s2 = fma(X[k + j * kLd], T[k + i * kLd], s2);
    }
    const double v = 0.5 * (s1 + s2);
    sK[i + j * kLd] = v;
    sK[j + i * kLd] = v;
  }
  __syncthreads();
  double* sZ = sH;  // H is no longer needed; T is free until V1 is formed
  const int sweeps = jacobi_eig<kThreads>(sK, T, sZ, L, lam, perm, sh, &flag);
  if (t == 0) {
    int r, sat;
    double kept;
    decide_rank(a, lam, L, snormC2, *a.normA2, &r, &sat, &kept);
    sr = r; ssat = sat; skept = kept;
  }
  __syncthreads();
  const int r = sr;
  // V1 = X Z_r (into T)
  for (int e = t; e < n * r; e += kThreads) {
    const int i = e % n, c = e / n;
    const int pc = perm[c];
    double s = 0.0;
    for (int k = 0; k < L; ++k) s = fma(X[i + k * kLd], sZ[k + pc * kLd], s);
    T[i + c * kLd] = s;
  }
  __syncthreads();
  canonical_signs<kThreads>(T, 1, kLd, n, r, sg);
  for (int e = t; e < n * r; e += kThreads) {
    const int i = e % n, c = e / n;
    const double v = T[i + c * kLd] * sg[c];
    a.V1[(int64_t)i * r + c] = v;
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
    rec->rho2 = 0.0;
    rec->sweeps = sweeps;
  }
  for (int i = t; i < kCMax; i += kThreads) a.rec->lam[i] = (i < L) ? lam[i] : 0.0;
}

// --------------------------------------------------------------------------
// X = orth(M) for n x c blocks (M column-major, X k-major).
// Register-resident variant for n <= R * tpj (one kernel per R so that each
// allocates only the registers it needs).
// (vall: the c reflectors of R * TPJ rows, c <= kThreads / TPJ)
template <int R, int TPJ>
__global__ __launch_bounds__(kThreads) void k_orth_reg(const double* M, double* X, int n, int c) {
  __shared__ double vbuf[2 * R * TPJ + kCMax];
  __shared__ double vall[R * kThreads];
  householder_reg<R, TPJ>(M, 1, n, X, c, 1, n, c, vbuf, nullptr, 0, 0, vall);
}

template <int R>
static void launch_orth_reg(double* M, double* X, int n, int c, hipStream_t st) {
  const int tpj = reg_group_width(c);
  if (tpj == 16) TT_LAUNCH((k_orth_reg<R, 16>), dim3(1), dim3(kThreads), 0, st, M, X, n, c);
  else if (tpj == 32) TT_LAUNCH((k_orth_reg<R, 32>), dim3(1), dim3(kThreads), 0, st, M, X, n, c);
  else TT_LAUNCH((k_orth_reg<R, 64>), dim3(1), dim3(kThreads), 0, st, M, X, n, c);
}

// --------------------------------------------------------------------------
// Rayleigh-Ritz on span(X) from K = Y^T Y (Y = A X): eigen-decomposition
// K = Z diag(lam) Z^T, rank decision, V1 = X Z_r (core side), W = Z_r so that
// the carry A V1 equals Y W.
constexpr int kRRThreads = 1024;  // measured: 16 waves finish a Jacobi round faster than 4
static_assert(kRRThreads == kThreads, "block_sum and step_norm2 assume kThreads threads per block");

__global__ __launch_bounds__(kRRThreads) void k_rr_solve(const double* __restrict__ K,
                                                         const double* __restrict__ X, SolveArgs a) {
  __shared__ __align__(16) double sK[kCMax * kLd];
  __shared__ double sK2[kCMax * kLd];
  __shared__ double sZ[kCMax * kLd];
  __shared__ double lam[kCMax], sg[kCMax], sh[32];
  __shared__ int perm[kCMax], flag, sr, ssat;
  __shared__ double skept, snormC2;
  const int t = threadIdx.x;
  const int n = a.n;
  const int L = a.ell;
  for (int e = t; e < L * L; e += kRRThreads) {
    const int i = e % L, j = e / L;
    sK[i + j * kLd] = 0.5 * (K[i + (int64_t)L * j] + K[j + (int64_t)L * i]);
  }
  {
    const double nc2 = step_norm2(a, sh);
    if (t == 0) snormC2 = nc2;
  }
  __syncthreads();
  const int sweeps = jacobi_eig<kRRThreads>(sK, sK2, sZ, L, lam, perm, sh, &flag);
  if (t == 0) {
    int r, sat;
    double kept;
    decide_rank(a, lam, L, snormC2, *a.normA2, &r, &sat, &kept);
    sr = r; ssat = sat; skept = kept;
  }
  __syncthreads();
  const int r = sr;
  // Z_r in eigenvalue order, k-major with an even row stride, in the (now
  // free) K buffer; a task is one row of V1 = X Z_r and eight of its columns,
  // the tasks of a wave share their columns (broadcast LDS reads) and each
  // output sums over k in order
  const int rp = (r + 1) & ~1;
  double* Zr = sK;
  for (int e = t; e < L * rp; e += kRRThreads) {
    const int k = e / rp, c = e % rp;
    Zr[e] = c < r ? sZ[k + perm[c] * kLd] : 0.0;
  }
  __syncthreads();
  const int nch = (r + 7) >> 3;
  for (int64_t task = t; task < (int64_t)n * nch; task += kRRThreads) {
    const int ch = (int)(task / n), i = (int)(task - (int64_t)ch * n);
    const int c0 = 8 * ch, cn = min(8, r - c0);
    const double* xr = X + (int64_t)i * L;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k = 0; k < L; ++k) {
      const double xk = xr[k];
      const double2* z = reinterpret_cast<const double2*>(Zr + k * rp + c0);   // within sK: k * rp + c0 + 8 <= 64 * 64 + 8
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double2 zz = z[j];
        acc[2 * j] = fma(xk, zz.x, acc[2 * j]);
        acc[2 * j + 1] = fma(xk, zz.y, acc[2 * j + 1]);
      }
    }
    double* out = a.V1 + (int64_t)i * r + c0;   // k-major: V1[i * r + c]
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < cn) out[j] = acc[j];
  }
  __threadfence_block();
  __syncthreads();
  canonical_signs<kRRThreads>(a.V1, r, 1, n, r, sg);
  const int64_t nr = (int64_t)n * r;
  for (int64_t e0 = t; e0 < nr; e0 += 4 * kRRThreads) {
    double vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = e0 + (int64_t)u * kRRThreads;
      vv[u] = e < nr ? a.V1[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = e0 + (int64_t)u * kRRThreads;
      if (e < nr) {
        const int i = (int)(e / r), c = (int)(e % r);
        const double v = vv[u] * sg[c];
        a.V1[e] = v;
        if (a.core) {
          if (a.core_layout == 0) a.core[i + (int64_t)n * c] = v;
          else a.core[c + (int64_t)r * i] = v;
        }
      }
    }
  }
  for (int e = t; e < L * r; e += kRRThreads) {
    const int k = e / r, c = e % r;
    a.W[(int64_t)k * r + c] = sZ[k + perm[c] * kLd] * sg[c];   // k-major
  }
  if (t == 0) {
    StepRec* rec = a.rec;
    rec->normC2 = snormC2;
    rec->kept2 = skept;
    rec->r = r;
    rec->sat = ssat;
    rec->ell = L;
    rec->resid2 = -1.0;
    rec->rho2 = 0.0;
    rec->sweeps = sweeps;
  }
  for (int i = t; i < kCMax; i += kRRThreads) a.rec->lam[i] = (i < L) ? lam[i] : 0.0;
}

// --------------------------------------------------------------------------
// Alg. 4 (ULV, right-to-left): range-side factorisation C ~ U L V^T with
// U^T E = 0.  U is an orthonormal basis of Y = C X, found on the long side by
// two rounds of an eigen-based Cholesky-QR: K = Y^T Y = P Lambda P^T,
// T = P Lambda^{-1/2}, Y <- Y T.  Directions with Lambda at or below
// 1e-14 Lambda_max (outside the numerical span) get a zero column; the
// second round restores orthonormality lost to K's rounding.  Then
// B^T = C^T U (one pass over C), B B^T = W S^2 W^T, V1 = B^T W_r S_r^{-1}
// (core side) and the carry U W_r S_r (the part of C outside span(U), the
// U2 L21 term, is not carried).
//
// k_alg4_basis: T (ell x ell, k-major: T(i,j) at i*ell + j) from K.
__global__ __launch_bounds__(kRRThreads) void k_alg4_basis(const double* __restrict__ K,
                                                           double* __restrict__ Tout, int L) {
  __shared__ double sK[kCMax * kLd];
  __shared__ double sK2[kCMax * kLd];
  __shared__ double sZ[kCMax * kLd];
  __shared__ double lam[kCMax], sh[32];
  __shared__ int perm[kCMax], flag;
  const int t = threadIdx.x;
  for (int e = t; e < L * L; e += kRRThreads) {
    const int i = e % L, j = e / L;
    sK[i + j * kLd] = 0.5 * (K[i + (int64_t)L * j] + K[j + (int64_t)L * i]);
  }
  __syncthreads();
  jacobi_eig<kRRThreads>(sK, sK2, sZ, L, lam, perm, sh, &flag);
  const double lmax = fmax(lam[0], 0.0);
  for (int e = t; e < L * L; e += kRRThreads) {
    const int i = e / L, j = e % L;
    const double lj = lam[j];
    Tout[e] = (lj > 1e-14 * lmax && lj > 0.0) ? sZ[i + perm[j] * kLd] / sqrt(lj) : 0.0;
  }
}

// k_alg4_solve: from E = Bt^T Bt (ell x ell) and Bt = C^T U (n x ell,
// column-major): rank, V1 = Bt W_r S_r^{-1} (canonical signs), core, carry
// weights W_r S_r (ell x r k-major, into a.W; carry = U a.W).
__global__ __launch_bounds__(kRRThreads) void k_alg4_solve(const double* __restrict__ E,
                                                           const double* __restrict__ Bt, SolveArgs a) {
  __shared__ double sE[kCMax * kLd];
  __shared__ double sK2[kCMax * kLd];
  __shared__ double sW[kCMax * kLd];
  __shared__ double lam[kCMax], sg[kCMax], sinv[kCMax], sh[32];
  __shared__ int perm[kCMax], flag, sr, ssat;
  __shared__ double skept, snormC2;
  const int t = threadIdx.x;
  const int n = a.n;
  const int L = a.ell;
  for (int e = t; e < L * L; e += kRRThreads) {
    const int i = e % L, j = e / L;
    sE[i + j * kLd] = 0.5 * (E[i + (int64_t)L * j] + E[j + (int64_t)L * i]);
  }
  {
    const double nc2 = step_norm2(a, sh);
    if (t == 0) snormC2 = nc2;
  }
  __syncthreads();
  const int sweeps = jacobi_eig<kRRThreads>(sE, sK2, sW, L, lam, perm, sh, &flag);
  if (t == 0) {
    int r, sat;
    double kept;
    decide_rank(a, lam, L, snormC2, *a.normA2, &r, &sat, &kept);
    sr = r; ssat = sat; skept = kept;
  }
  if (t < L) {
    const double sv = sqrt(fmax(lam[t], 0.0));
    sinv[t] = sv > 0.0 ? 1.0 / sv : 0.0;
  }
  __syncthreads();
  const int r = sr;
  for (int64_t e = t; e < (int64_t)n * r; e += kRRThreads) {
    const int i = (int)(e / r), c = (int)(e % r);
    const int pc = perm[c];
    double s = 0.0;
    for (int k = 0; k < L; ++k) s = fma(Bt[i + (int64_t)n * k], sW[k + pc * kLd], s);
    a.V1[e] = s * sinv[c];
  }
  __threadfence_block();
  __syncthreads();
  canonical_signs<kRRThreads>(a.V1, r, 1, n, r, sg);
  const int64_t nr = (int64_t)n * r;
  for (int64_t e0 = t; e0 < nr; e0 += 4 * kRRThreads) {
    double vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = e0 + (int64_t)u * kRRThreads;
      vv[u] = e < nr ? a.V1[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = e0 + (int64_t)u * kRRThreads;
      if (e < nr) {
        const int i = (int)(e / r), c = (int)(e % r);
        const double v = vv[u] * sg[c];
        a.V1[e] = v;
        if (a.core) {
          if (a.core_layout == 0) a.core[i + (int64_t)n * c] = v;
          else a.core[c + (int64_t)r * i] = v;
        }
      }
    }
  }
  for (int e = t; e < L * r; e += kRRThreads) {
    const int k = e / r, c = e % r;
    a.W[(int64_t)k * r + c] = sW[k + perm[c] * kLd] * sqrt(fmax(lam[c], 0.0)) * sg[c];
  }
  if (t == 0) {
    StepRec* rec = a.rec;
    rec->normC2 = snormC2;
    rec->kept2 = skept;
    rec->r = r;
    rec->sat = ssat;
    rec->ell = L;
    rec->resid2 = -1.0;
    rec->rho2 = 0.0;
    rec->sweeps = sweeps;
  }
  for (int i = t; i < kCMax; i += kRRThreads) a.rec->lam[i] = (i < L) ? lam[i] : 0.0;
}

// --------------------------------------------------------------------------
// Deflation inner kernel: one core-side vector at a time (the USV-plus reading
// of the paper's fastest TT-ULV variant, Sec. 3.3 / Sec. 4).  Vector j starts
// from column j of the step's Gaussian test matrix with the vectors found so
// far projected out, takes q power steps x <- P(A^T A x) / ||P(A^T A x)|| (a
// step whose product vanishes keeps x), and adds its energy ||A v_j||^2 to the
// kept energy; the search ends at the fixed rank, at the first j with
// ||C||^2 - kept <= eps_k^2 (the rank rule after Alg. 2), or after cap vectors.
// P is two rounds of classical Gram-Schmidt, z <- z - V (V^T z).

// z <- z - V (V^T z) over the first j columns of V (LDS, column l at V + l kLd),
// n <= 64, two rounds.  cbuf holds kCMax coefficients.
__device__ __forceinline__ void defl_project_lds(double* z, const double* V, int n, int j, double* cbuf) {
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const int row = t >> 4, p = t & 15;
  for (int round = 0; round < 2 && j > 0; ++round) {
    for (int l = wv; l < j; l += kThreads / 64) {
      const double v = lane < n ? V[lane + l * kLd] * z[lane] : 0.0;
      const double c = group_sum(v, 64);
      if (lane == 0) cbuf[l] = c;
    }
    __syncthreads();
    double sacc = 0.0;
    if (row < n)
      for (int l = p; l < j; l += 16) sacc = fma(V[row + l * kLd], cbuf[l], sacc);
    sacc = row16_sum(sacc);
    if (row < n && p == 0) z[row] -= sacc;   // z's readers above finished at the barrier
    __syncthreads();
  }
}

// ||z||^2 for z in LDS, n <= 64: the same value in every thread.
__device__ __forceinline__ double defl_norm2_lds(const double* z, int n, double* sh) {
  const int t = threadIdx.x;
  if (t < 64) {
    const double v = t < n ? z[t] * z[t] : 0.0;
    const double s2 = group_sum(v, 64);
    if (t == 0) sh[0] = s2;
  }
  __syncthreads();
  const double s2 = sh[0];
  __syncthreads();
  return s2;
}

// y = H x, H held in registers: thread (row, p) keeps H(row, p + 16 u), u < 4.
__device__ __forceinline__ void defl_matvec(const double (&h)[4], const double* x, double* y, int n) {
  const int t = threadIdx.x, row = t >> 4, p = t & 15;
  double sacc = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = p + 16 * u;
    if (k < n) sacc = fma(h[u], x[k], sacc);
  }
  sacc = row16_sum(sacc);
  if (row < n && p == 0) y[row] = sacc;
  __syncthreads();
}

// Column j of the step's test matrix with the first j columns of V projected
// out, normalised, into x (LDS).
__device__ __forceinline__ void defl_start_lds(const SolveArgs& a, int j, double* x, const double* V, int n,
                                               double* cbuf, double* sh) {
  if (threadIdx.x < n) x[threadIdx.x] = sketch_row_entry(a, threadIdx.x, j);
  __syncthreads();
  defl_project_lds(x, V, n, j, cbuf);
  const double nx = sqrt(defl_norm2_lds(x, n, sh));
  if (threadIdx.x < n && nx > 0.0) x[threadIdx.x] = x[threadIdx.x] / nx;
  __syncthreads();
}

// Writes V1 = V[:, :r] with canonical column signs (k-major, i r + c) and the
// core in its layout; V (column-major, column stride ldv) may be in LDS or
// global memory.
__device__ __forceinline__ void defl_write_basis(const SolveArgs& a, const double* V, int64_t ldv, int n, int r,
                                                 double* sg) {
  canonical_signs<kThreads>(V, 1, ldv, n, r, sg);
  const int64_t nr = (int64_t)n * r;
  for (int64_t e = threadIdx.x; e < nr; e += kThreads) {
    const int i = (int)(e / r), c = (int)(e % r);
    const double v = V[i + c * ldv] * sg[c];
    a.V1[e] = v;
    if (a.core) {
      if (a.core_layout == 0) a.core[i + (int64_t)n * c] = v;
      else a.core[c + (int64_t)r * i] = v;
    }
  }
}

// Gram mode: H = A^T A (n x n column-major, n <= 64), the whole search in one
// workgroup; ||C||^2 = trace(H).
__global__ __launch_bounds__(kThreads) void k_defl_gram(const double* __restrict__ H, SolveArgs a, int cap) {
  __shared__ double sV[kCMax * kLd];
  __shared__ double sx[kCMax], sz[kCMax], cbuf[kCMax], lam[kCMax], sg[kCMax], sh[32];
  __shared__ double snc2;
  const int t = threadIdx.x, n = a.n;
  const int row = t >> 4, p = t & 15;
  double h[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = p + 16 * u;
    h[u] = (row < n && k < n) ? H[row + (int64_t)n * k] : 0.0;
  }
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += H[i + (int64_t)n * i];
    snc2 = tr;
    if (a.first) *a.normA2 = tr;
  }
  __syncthreads();
  const double normC2 = snc2;
  const double eps2 = a.eps_factor2 * (a.first ? normC2 : *a.normA2);
  double kept = 0.0;
  int r = 0, sat = a.r_fixed > 0 ? 1 : 0;
  for (int j = 0; j < cap; ++j) {
    defl_start_lds(a, j, sx, sV, n, cbuf, sh);
    for (int it = 0; it < a.q; ++it) {
      defl_matvec(h, sx, sz, n);
      defl_project_lds(sz, sV, n, j, cbuf);
      const double nz = sqrt(defl_norm2_lds(sz, n, sh));
      if (t < n && nz > 0.0) sx[t] = sz[t] / nz;
      __syncthreads();
    }
    if (t < n) sV[t + j * kLd] = sx[t];
    // energy x^T H x
    defl_matvec(h, sx, sz, n);
    if (t < 64) {
      const double v = t < n ? sx[t] * sz[t] : 0.0;
      const double e = group_sum(v, 64);
      if (t == 0) lam[j] = e;
    }
    __syncthreads();
    kept += lam[j];   // every thread keeps the same running sum
    r = j + 1;
    const bool stop = (a.r_fixed > 0) ? (r >= a.r_fixed) : (normC2 - kept <= eps2);
    if (stop) {
      if (a.r_fixed <= 0) sat = 1;
      break;
    }
  }
  __syncthreads();
  defl_write_basis(a, sV, kLd, n, r, sg);
  if (t == 0) {
    StepRec* rec = a.rec;
    rec->normC2 = normC2;
    rec->kept2 = kept;
    rec->r = r;
    rec->sat = sat;
    rec->ell = r;
    rec->resid2 = -1.0;
    rec->rho2 = 0.0;
    rec->sweeps = 0;
  }
  for (int i = t; i < kCMax; i += kThreads) a.rec->lam[i] = (i < r) ? lam[i] : 0.0;
}

// ---- tall mode: V (n x cap) and x in global memory, n <= 4096 -------------
// z <- z - V (V^T z) over the first j columns (z in LDS), two rounds: the
// coefficient of column l is one wave's sum, then thread i updates rows i,
// i + kThreads, ...  Up to n = 1024 a lane's loads go four at a time.  Wider
// vectors issue every load of a batch before the first use (16 rows of a
// column per lane, 16 columns of a row per thread; indices past n or j
// clamped and their values masked), so that the dependent memory round trips
// per round fall from about n/256 + 4 ceil(j/4) to n/1024 + 4 ceil(j/16).
__device__ __forceinline__ void defl_project_global(double* z, const double* V, int n, int j, double* cbuf) {
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const bool wide = n > kThreads;
  for (int round = 0; round < 2 && j > 0; ++round) {
    for (int l = wv; l < j; l += kThreads / 64) {
      const double* v = V + (int64_t)l * n;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (wide) {
        for (int i0 = lane; i0 < n; i0 += 64 * 16) {
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int i = i0 + 64 * u;
            const int ic = i < n ? i : n - 1;
            acc[u & 3] = fma(v[ic], i < n ? z[ic] : 0.0, acc[u & 3]);
          }
        }
      } else {
        for (int i0 = lane; i0 < n; i0 += 256) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + 64 * u;
            if (i < n) acc[u] = fma(v[i], z[i], acc[u]);
          }
        }
      }
      const double c = group_sum((acc[0] + acc[1]) + (acc[2] + acc[3]), 64);
      if (lane == 0) cbuf[l] = c;
    }
    __syncthreads();
    for (int i = t; i < n; i += kThreads) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (wide) {
        for (int l0 = 0; l0 < j; l0 += 16) {
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int l = l0 + u;
            const int lc = l < j ? l : j - 1;
            acc[u & 3] = fma(V[i + (int64_t)lc * n], l < j ? cbuf[lc] : 0.0, acc[u & 3]);
          }
        }
      } else {
        int l = 0;
        for (; l + 4 <= j; l += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] = fma(V[i + (int64_t)(l + u) * n], cbuf[l + u], acc[u]);
        }
        for (; l < j; ++l) acc[0] = fma(V[i + (int64_t)l * n], cbuf[l], acc[0]);
      }
      z[i] -= (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ double defl_norm2_global(const double* z, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) v = fma(z[i], z[i], v);
  return block_sum(v, sh);
}

// x <- column j of the test matrix, projected and normalised (LDS staging zs).
__device__ __forceinline__ void defl_start_global(const DeflArgs& d, int j, double* zs, double* cbuf, double* sh) {
  const int n = d.a.n;
  for (int i = threadIdx.x; i < n; i += kThreads) zs[i] = sketch_row_entry(d.a, i, j);
  __syncthreads();
  defl_project_global(zs, d.V, n, j, cbuf);
  const double nx = sqrt(defl_norm2_global(zs, n, sh));
  for (int i = threadIdx.x; i < n; i += kThreads) d.x[i] = nx > 0.0 ? zs[i] / nx : zs[i];
}

__global__ __launch_bounds__(kThreads) void k_defl_start(DeflArgs d) {
  __shared__ double zs[kDeflMaxN], cbuf[kCMax], sh[32];
  if (threadIdx.x == 0) {
    d.st->normC2 = 0.0;
    d.st->kept = 0.0;
    d.st->r = 0;
    d.st->sat = d.a.r_fixed > 0 ? 1 : 0;
    d.st->done = 0;
  }
  for (int i = threadIdx.x; i < kCMax; i += kThreads) d.a.rec->lam[i] = 0.0;
  defl_start_global(d, 0, zs, cbuf, sh);
}

// The kept vectors' bookkeeping after the energy ||A v_{j-1}||^2 = e is known
// (thread 0): returns whether the search ends here.
__device__ __forceinline__ bool defl_account(const DeflArgs& d, int j, double e) {
  DeflState* S = d.st;
  const double kept = S->kept + e;
  S->kept = kept;
  S->r = j;
  d.a.rec->lam[j - 1] = e;
  const double eps2 = d.a.eps_factor2 * (*d.a.normA2);
  const bool stop = (d.a.r_fixed > 0) ? (j >= d.a.r_fixed) : (S->normC2 - kept <= eps2);
  if (stop || j >= d.cap) {
    S->done = 1;
    if (d.a.r_fixed <= 0) S->sat = stop ? 1 : 0;
  }
  return S->done != 0;
}

// After a pass over the iterate x (and, with has_w, over the finished vector
// v_{j-1}): account v_{j-1}, then the power step of vector j; finish: vector j
// is complete, stored, and vector j + 1 is started.
__global__ __launch_bounds__(kThreads) void k_defl_update(const double* __restrict__ zr, DeflArgs d, int j, int has_w,
                                                          int finish, int first_pass) {
  __shared__ double zs[kDeflMaxN], cbuf[kCMax], sh[32];
  __shared__ int sdone;
  const int t = threadIdx.x, n = d.a.n;
  if (t == 0) {
    DeflState* S = d.st;
    int done = S->done;
    if (!done && first_pass) {
      S->normC2 = zr[n + 2];
      if (d.a.first) *d.a.normA2 = zr[n + 2];
    }
    if (!done && has_w) done = defl_account(d, j, zr[n + 1]);
    sdone = done;
  }
  __syncthreads();
  if (sdone) return;
  for (int i = t; i < n; i += kThreads) zs[i] = zr[i];
  __syncthreads();
  defl_project_global(zs, d.V, n, j, cbuf);
  const double nz = sqrt(defl_norm2_global(zs, n, sh));
  double* vj = d.V + (int64_t)j * n;
  for (int i = t; i < n; i += kThreads) {
    const double xi = nz > 0.0 ? zs[i] / nz : d.x[i];
    d.x[i] = xi;
    if (finish) vj[i] = xi;
  }
  if (finish && j + 1 < d.cap) {
    __threadfence_block();   // column j of V is written before the next start vector reads it
    __syncthreads();
    defl_start_global(d, j + 1, zs, cbuf, sh);
  }
}

// The energy of the last vector (a pass over w = v_{cap-1} alone).
__global__ void k_defl_last(const double* __restrict__ zr, DeflArgs d) {
  if (threadIdx.x != 0 || d.st->done) return;
  defl_account(d, d.cap, zr[d.a.n + 1]);
}

__global__ __launch_bounds__(kThreads) void k_defl_finish(DeflArgs d) {
  __shared__ double sg[kCMax];
  const DeflState* S = d.st;
  const int r = S->r;
  defl_write_basis(d.a, d.V, d.a.n, d.a.n, r, sg);
  if (threadIdx.x == 0) {
    StepRec* rec = d.a.rec;
    rec->normC2 = S->normC2;
    rec->kept2 = S->kept;
    rec->r = r;
    rec->sat = S->sat;
    rec->ell = r;
    rec->resid2 = -1.0;
    rec->rho2 = 0.0;
    rec->sweeps = 0;
  }
}

}  // namespace

hipError_t launch_defl_gram(const double* H, const SolveArgs& a, int cap, hipStream_t st) {
  if (a.n < 1 || a.n > kGramMax || cap < 1 || cap > a.n || cap > kCMax || a.q < 1) return hipErrorInvalidValue;
  TT_LAUNCH(k_defl_gram, dim3(1), dim3(kThreads), 0, st, H, a, cap);
  return hipGetLastError();
}

static bool defl_args_ok(const DeflArgs& d) {
  return d.a.n >= 1 && d.a.n <= kDeflMaxN && d.cap >= 1 && d.cap <= kCMax && d.cap <= d.a.n && d.V && d.x && d.st;
}

hipError_t launch_defl_start(const DeflArgs& d, hipStream_t st) {
  if (!defl_args_ok(d)) return hipErrorInvalidValue;
  TT_LAUNCH(k_defl_start, dim3(1), dim3(kThreads), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_defl_update(const double* zr, const DeflArgs& d, int j, int has_w, int finish, int first_pass,
                              hipStream_t st) {
  if (!defl_args_ok(d) || j < 0 || j >= d.cap || (has_w && j < 1)) return hipErrorInvalidValue;
  TT_LAUNCH(k_defl_update, dim3(1), dim3(kThreads), 0, st, zr, d, j, has_w, finish, first_pass);
  return hipGetLastError();
}

hipError_t launch_defl_last(const double* zr, const DeflArgs& d, hipStream_t st) {
  if (!defl_args_ok(d)) return hipErrorInvalidValue;
  TT_LAUNCH(k_defl_last, dim3(1), dim3(64), 0, st, zr, d);
  return hipGetLastError();
}

hipError_t launch_defl_finish(const DeflArgs& d, hipStream_t st) {
  if (!defl_args_ok(d)) return hipErrorInvalidValue;
  TT_LAUNCH(k_defl_finish, dim3(1), dim3(kThreads), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_gram_solve(const double* H, const SolveArgs& a, hipStream_t st) {
  if (a.n < 1 || a.n > kGramMax || a.ell < 1) return hipErrorInvalidValue;
  TT_LAUNCH(k_gram_solve, dim3(1), dim3(kThreads), 0, st, H, a);
  return hipGetLastError();
}

hipError_t launch_gen_sketch(double* G, const SolveArgs& a, hipStream_t st) {
  const int64_t total = (int64_t)a.n * a.ell;
  if (total < 1) return hipErrorInvalidValue;
  TT_LAUNCH(k_gen_sketch, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, G, a);
  return hipGetLastError();
}

// Taller blocks: a tree of register QRs (TSQR).  The n rows are split into P
// balanced leaf blocks of at most tsqr_block_rows(c) rows (each at least half
// that, so never fewer than c); leaf b factors M_b = Q_b R_b in its own
// workgroup, Q_b overwriting its rows of M and R_b going to rows b*c .. b*c+c-1
// of the stacked (P c) x c matrix S.  Then S = Q_S R (recursively, by the same
// routine), and X = diag(Q_b) Q_S: row i of leaf b is Q_b(i, :) Q_S(b c : b c + c, :).
// X spans the column space of M and has orthonormal columns like the one-block
// factorisation (the two may differ in the signs of the columns).
static int tsqr_block_rows(int c) { return 16 * reg_group_width(c); }

__host__ __device__ __forceinline__ void tsqr_block(int n, int P, int b, int* r0, int* rows) {
  const int q = n / P, e = n % P;   // the first e blocks take one more row
  *r0 = b * q + (b < e ? b : e);
  *rows = q + (b < e ? 1 : 0);
}

template <int R, int TPJ>
__global__ __launch_bounds__(kThreads) void k_tsqr_leaf(double* M, int n, int c, int P, double* S) {
  __shared__ double vbuf[2 * R * TPJ + kCMax];
  __shared__ double vall[R * kThreads];
  int r0, rows;
  tsqr_block(n, P, blockIdx.x, &r0, &rows);
  householder_reg<R, TPJ>(M + r0, 1, n, M + r0, 1, n, rows, c, vbuf, S + (int64_t)blockIdx.x * c, 1,
                          (int64_t)P * c, vall);
}

constexpr int kCombineThreads = 256;
__global__ __launch_bounds__(kCombineThreads) void k_tsqr_combine(const double* __restrict__ M, int n, int c, int P,
                                                                  const double* __restrict__ QS, double* __restrict__ X) {
  __shared__ double sq[kCMax * kCMax];
  int r0, rows;
  tsqr_block(n, P, blockIdx.x, &r0, &rows);
  // rows b*c .. b*c+c-1 of Q_S (k-major) are one contiguous c x c block
  for (int e = threadIdx.x; e < c * c; e += kCombineThreads) sq[e] = QS[(int64_t)blockIdx.x * c * c + e];
  __syncthreads();
  for (int e = threadIdx.x; e < rows * c; e += kCombineThreads) {
    const int i = e / c, j = e % c;
    double s = 0.0;
    for (int l = 0; l < c; ++l) s = fma(M[(r0 + i) + (int64_t)l * n], sq[l * c + j], s);
    X[(int64_t)(r0 + i) * c + j] = s;
  }
}

template <int R>
static void launch_tsqr_leaf(double* M, int n, int c, int P, double* S, hipStream_t st) {
  const int tpj = reg_group_width(c);
  if (tpj == 16) TT_LAUNCH((k_tsqr_leaf<R, 16>), dim3(P), dim3(kThreads), 0, st, M, n, c, P, S);
  else if (tpj == 32) TT_LAUNCH((k_tsqr_leaf<R, 32>), dim3(P), dim3(kThreads), 0, st, M, n, c, P, S);
  else TT_LAUNCH((k_tsqr_leaf<R, 64>), dim3(P), dim3(kThreads), 0, st, M, n, c, P, S);
}

int64_t orth_scratch(int n, int c) {
  if (c < 1 || c > kCMax || n <= tsqr_block_rows(c)) return 0;
  const int P = (n + tsqr_block_rows(c) - 1) / tsqr_block_rows(c);
  const int n2 = P * c;
  return 2 * (int64_t)n2 * c + orth_scratch(n2, c);
}

hipError_t launch_orth(double* M, double* X, int n, int c, double* scratch, int64_t scratch_len, hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || c > n) return hipErrorInvalidValue;
  const int nbmax = tsqr_block_rows(c);
  if (n <= nbmax) {
    switch (reg_rows(n, c)) {
      case 4: launch_orth_reg<4>(M, X, n, c, st); break;
      case 8: launch_orth_reg<8>(M, X, n, c, st); break;
      default: launch_orth_reg<16>(M, X, n, c, st); break;
    }
    return hipGetLastError();
  }
  if (!scratch || scratch_len < orth_scratch(n, c)) return hipErrorInvalidValue;
  const int P = (n + nbmax - 1) / nbmax;
  const int n2 = P * c;
  double* S = scratch;
  double* QS = scratch + (int64_t)n2 * c;
  const int rmax = (n + P - 1) / P;   // rows of the largest leaf block
  switch (reg_rows(rmax, c)) {
    case 4: launch_tsqr_leaf<4>(M, n, c, P, S, st); break;
    case 8: launch_tsqr_leaf<8>(M, n, c, P, S, st); break;
    default: launch_tsqr_leaf<16>(M, n, c, P, S, st); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_orth(S, QS, n2, c, QS + (int64_t)n2 * c, scratch_len - 2 * (int64_t)n2 * c, st);
  if (e != hipSuccess) return e;
  TT_LAUNCH(k_tsqr_combine, dim3(P), dim3(kCombineThreads), 0, st, M, n, c, P, QS, X);
  return hipGetLastError();
}

hipError_t launch_rr_solve(const double* K, const double* X, const SolveArgs& a, hipStream_t st) {
  if (a.n < 1 || a.ell < 1 || a.ell > kCMax) return hipErrorInvalidValue;
  TT_LAUNCH(k_rr_solve, dim3(1), dim3(kRRThreads), 0, st, K, X, a);
  return hipGetLastError();
}

}  // namespace ttutv

namespace ttutv {
hipError_t launch_alg4_basis(const double* K, double* T, int ell, hipStream_t st) {
  if (ell < 1 || ell > kCMax) return hipErrorInvalidValue;
  TT_LAUNCH(k_alg4_basis, dim3(1), dim3(kRRThreads), 0, st, K, T, ell);
  return hipGetLastError();
}
hipError_t launch_alg4_solve(const double* E, const double* Bt, const SolveArgs& a, hipStream_t st) {
  if (a.n < 1 || a.ell < 1 || a.ell > kCMax) return hipErrorInvalidValue;
  TT_LAUNCH(k_alg4_solve, dim3(1), dim3(kRRThreads), 0, st, E, Bt, a);
  return hipGetLastError();
}
}  // namespace ttutv

namespace ttutv {

// ---- shifted CholeskyQR3 orthonormalisation --------------------------------
// X = orth(M) for M n x c (column-major), c <= 64, by three shifted
// Cholesky-QR rounds: Q <- Q R^{-1} with R^T R = Q^T Q + s I, starting from Q
// = M.  The shift s = 11 (n c + c (c + 1)) u tr(Q^T Q) (tr bounds ||Q||_2^2
// from above) keeps each factorisation positive definite for condition
// numbers up to about 1/u, and each round takes the condition number of Q to
// about its square root (the shifted CholeskyQR of Fukaya, Kannan,
// Nakatsukasa, Yamamoto and Yanagisawa, SIAM J. Sci. Comput. 2020, whose
// CholeskyQR3 shifts only the first round).  The later rounds are shifted too
// so that an exactly rank-deficient iterate (an exact-rank tensor sketched
// wider than its rank) stays finite: its dead directions, scaled up round by
// round, end as further orthonormal columns.  The result is orthonormal to
// about the shift's size rather than to rounding, which suffices for the
// intermediate power iterates it is used for (the last iterate, which feeds
// the Rayleigh-Ritz step, takes Householder QR).  The Gram matrices go
// through the streaming Gram kernel; each factorisation is one wave.
namespace {

// One wave: K (c x c, column-major) + shift I = R^T R (R upper), then Rinv =
// R^{-1} (c x c column-major) to global.  Lane l carries column l of the
// trailing matrix in registers; row j of R is broadcast through LDS.
template <int CM>
__global__ __launch_bounds__(64) void k_chol_inv(const double* __restrict__ K, double* __restrict__ Rinv, int c,
                                                 double shift_factor) {
  __shared__ double sR[CM][CM + 2];
  const int l = threadIdx.x;
  double k[CM];
#pragma unroll
  for (int i = 0; i < CM; ++i) k[i] = (i < c && l < c) ? K[i + (int64_t)c * l] : 0.0;
  if (shift_factor > 0.0) {
    // trace of K: lane l holds K(l, l) in k[l]; summed in a fixed order through LDS
    double dl = 0.0;
#pragma unroll
    for (int i = 0; i < CM; ++i)
      if (i == l) dl = k[i];
    if (l < c) sR[0][l] = dl;
    __syncthreads();
    double tr = 0.0;
    for (int i = 0; i < c; ++i) tr += sR[0][i];
    __syncthreads();
    const double s = shift_factor * tr;
#pragma unroll
    for (int i = 0; i < CM; ++i)
      if (i == l && l < c) k[i] += s;
  }
  for (int j = 0; j < c; ++j) {
    // pivot K(j, j), held by lane j
    double kjl = 0.0;
#pragma unroll
    for (int i = 0; i < CM; ++i)
      if (i == j) kjl = k[i];
    if (l == j) sR[j][CM + 1] = kjl;
    __syncthreads();
    const double dj = sR[j][CM + 1];
    // a non-positive pivot (only for non-finite or exactly singular input
    // beyond the shift) is replaced by the smallest normal number
    const double piv = dj > 0.0 ? sqrt(dj) : 2.2250738585072014e-308;
    if (l < CM) sR[j][l] = (l >= j && l < c) ? kjl / piv : 0.0;   // R(j, l)
    __syncthreads();
    double rj[CM];
#pragma unroll
    for (int i = 0; i < CM; ++i) rj[i] = sR[j][i];
    const double rjl = (l < CM) ? sR[j][l] : 0.0;
#pragma unroll
    for (int i = 0; i < CM; ++i)
      if (i > j) k[i] = fma(-rj[i], rjl, k[i]);
  }
  __syncthreads();
  // Rinv column l by back substitution on R (upper): R x = e_l
  double x[CM];
#pragma unroll
  for (int i = CM - 1; i >= 0; --i) {
    double v = (i == l) ? 1.0 : 0.0;
    if (i < c) {
#pragma unroll
      for (int p = i + 1; p < CM; ++p)
        if (p < c) v = fma(-sR[i][p], x[p], v);
      v /= sR[i][i];
    } else {
      v = 0.0;
    }
    x[i] = v;
  }
  if (l < c) {
#pragma unroll
    for (int i = 0; i < CM; ++i)
      if (i < c) Rinv[i + (int64_t)c * l] = x[i];
  }
}

// X = M Rinv row by row (Rinv c x c upper, in LDS): one row per thread.  M and
// X column-major (COL) or k-major (row-major, ROW).
template <int CM>
__global__ __launch_bounds__(256) void k_rows_rinv(const double* __restrict__ M, int m_row_major,
                                                   const double* __restrict__ Rinv, double* __restrict__ X,
                                                   int x_row_major, int n, int c) {
  __shared__ double sI[CM][CM + 1];
  for (int e = threadIdx.x; e < c * c; e += 256) sI[e % c][e / c] = Rinv[e];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  double m[CM];
#pragma unroll
  for (int j = 0; j < CM; ++j) m[j] = (j < c) ? M[m_row_major ? r * c + j : r + (int64_t)n * j] : 0.0;
  // fully unrolled (constant indices keep m in registers); columns past c
  // are skipped, not broken out of
#pragma unroll
  for (int j = 0; j < CM; ++j) {
    if (j < c) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i <= j; ++i) v = fma(m[i], sI[i][j], v);
      X[x_row_major ? r * c + j : r + (int64_t)n * j] = v;
    }
  }
}

template <int CM>
hipError_t cholqr_round(const double* src, int src_row_major, double* dst, int dst_row_major, int n, int c,
                        double shift_factor, double* K, double* Rinv, double* parts, hipStream_t st) {
  const int kch = atb_chunks(n, c, c);
  hipError_t e = launch_atb(src, 0, src, 0, n, c, c, src_row_major ? ROW : COL, kch == 1 ? K : parts, kch, st);
  if (e != hipSuccess) return e;
  if (kch > 1) {
    e = launch_reduce(parts, kch, (int64_t)c * c, K, nullptr, st);
    if (e != hipSuccess) return e;
  }
  TT_LAUNCH((k_chol_inv<CM>), dim3(1), dim3(64), 0, st, K, Rinv, c, shift_factor);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  TT_LAUNCH((k_rows_rinv<CM>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, src_row_major, Rinv, dst,
            dst_row_major, n, c);
  return hipGetLastError();
}

template <int CM>
hipError_t cholqr3(const double* M, double* X, int n, int c, double* scratch, hipStream_t st) {
  double* Q1 = scratch;
  double* Q2 = Q1 + (int64_t)n * c;
  double* K = Q2 + (int64_t)n * c;
  double* Rinv = K + (int64_t)c * c;
  double* parts = Rinv + (int64_t)c * c;
  const double shift = 11.0 * ((double)n * c + (double)c * (c + 1)) * ldexp(1.0, -53);
  hipError_t e = cholqr_round<CM>(M, 0, Q1, 0, n, c, shift, K, Rinv, parts, st);
  if (e == hipSuccess) e = cholqr_round<CM>(Q1, 0, Q2, 0, n, c, shift, K, Rinv, parts, st);
  if (e == hipSuccess) e = cholqr_round<CM>(Q2, 0, X, 1, n, c, shift, K, Rinv, parts, st);
  return e;
}

}  // namespace

int64_t orth_cholqr_scratch(int n, int c) {
  return 2 * (int64_t)n * c + 2 * (int64_t)c * c + (int64_t)atb_chunks(n, c, c) * c * c;
}

hipError_t launch_orth_cholqr(const double* M, double* X, int n, int c, double* scratch, int64_t scratch_len,
                              hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || c > n) return hipErrorInvalidValue;
  if (!scratch || scratch_len < orth_cholqr_scratch(n, c)) return hipErrorInvalidValue;
  if (c <= 16) return cholqr3<16>(M, X, n, c, scratch, st);
  if (c <= 32) return cholqr3<32>(M, X, n, c, scratch, st);
  return cholqr3<64>(M, X, n, c, scratch, st);
}

}  // namespace ttutv
