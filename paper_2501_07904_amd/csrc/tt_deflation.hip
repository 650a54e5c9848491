// The streaming pass of the deflation inner kernel (one core-side vector at a
// time, the USV-plus reading of Sec. 3.3 / Sec. 4): for the tall A (m x n) of
// a step and the current iterate x, z = A^T (A x) and ||A x||^2, together with
// the energy ||A w||^2 of the vector finished last and, on a step's first pass,
// ||A||_F^2 -- all from one read of A.  Each power step of the search costs one
// such pass (HBM-bound: 4 m n flops on m n elements).
//
// Each workgroup owns a contiguous band of rows and holds its share of z in
// registers: a thread keeps every 256th (four-wave form) or 64th (one-wave
// form) column, so z needs no reduction inside the band.  A band is read in
// chunks of RC rows (RC NC = 16 elements per thread, one row at least); the
// chunk's row products y = A x and A w need a sum over the workgroup, done for
// all 2 RC values together by a halving butterfly (each exchange step halves
// the values a lane holds), then, in the four-wave form, the four wave
// partials added in a fixed order, so every thread applies the same y.  The
// per-workgroup partials are summed in a fixed order by the reduction kernels.
#include "tt_internal.h"

namespace ttutv {

namespace {

constexpr int kPT = 256;       // threads per workgroup
constexpr int kPerThread = 16; // elements of A per thread and chunk (at least one row)
constexpr int kWaveMaxN = 512; // widest core side of the one-wave form (row-major A)
constexpr int kWaveMaxNCol = 128; // (column-major A: each lane then reads runs of at least 8 rows)

// Sums the V values of every lane over the 64 lanes of a wave.  Each halving
// step at lane distance O pairs a lane with lane ^ O: the lane without bit O
// keeps the sums of the lower half of its values, its partner those of the
// upper half; once one value is left, plain exchange steps finish the sum.  On
// return lane l holds the sum of value l >> (6 - log2 V) (the lanes holding one
// value hold bitwise-equal sums).
template <int CNT, int O, int V>
__device__ __forceinline__ void wave_multi_sum_step(double (&v)[V], int lane) {
  if constexpr (O >= 1) {
    if constexpr (CNT > 1) {
      constexpr int h = CNT / 2;
      const bool up = (lane & O) != 0;
#pragma unroll
      for (int k = 0; k < h; ++k) {
        const double send = up ? v[k] : v[k + h];
        const double keep = up ? v[k + h] : v[k];
        v[k] = keep + __shfl_xor(send, O, 64);
      }
      wave_multi_sum_step<h, O / 2, V>(v, lane);
    } else {
      v[0] += __shfl_xor(v[0], O, 64);
      wave_multi_sum_step<1, O / 2, V>(v, lane);
    }
  }
}

template <int V>
__device__ __forceinline__ double wave_multi_sum(double (&v)[V], int lane) {
  wave_multi_sum_step<V, 32, V>(v, lane);
  return v[0];
}

template <int V>
constexpr int log2c() {
  return V <= 1 ? 0 : 1 + log2c<V / 2>();
}

// Rows [i0, i0 + RC) of the band (ending at r1 >= 1) into registers; rows past
// the band and columns past n read as zero.  FULL: every row is inside the band,
// so the loads are unconditional (the column is clamped into A and the value
// masked), and all of a chunk's loads are issued before the first wait; the
// band's last, partial chunk checks its rows.
template <bool FULL, typename TA, int LY, int NC, int RC>
__device__ __forceinline__ void pass_load(const TA* __restrict__ A, int64_t m, int n, int64_t i0, int64_t r1,
                                          double (&a)[RC][NC]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int rr = 0; rr < RC; ++rr) {
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int64_t i = i0 + rr;
      const int col = t + kPT * u;
      const int cc = col < n ? col : n - 1;
      if (FULL) {
        const double v = (double)A[LY == COL ? i + (int64_t)cc * m : i * n + cc];
        a[rr][u] = col < n ? v : 0.0;
      } else {
        a[rr][u] = (i < r1 && col < n) ? (double)A[LY == COL ? i + (int64_t)cc * m : i * n + cc] : 0.0;
      }
    }
  }
}

// One chunk: the row products A x and A w summed over the workgroup (sred
// buffer `buf`, one barrier), then z += A^T (A x) on the thread's columns and
// the chunk's shares of ||A x||^2, ||A w||^2 and ||A||^2.
template <int NC, int RC>
__device__ __forceinline__ void pass_chunk(const double (&a)[RC][NC], const double (&xv)[NC], const double (&wvv)[NC],
                                           double (&z)[NC], double& ex, double& ew, double& sq, int want_sq,
                                           double (*sred)[2 * RC]) {
  constexpr int NV = 2 * RC;
  constexpr int SH = 6 - log2c<NV>();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double v[NV];
#pragma unroll
  for (int rr = 0; rr < RC; ++rr) {
    double px = 0.0, pw = 0.0;
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      px = fma(a[rr][u], xv[u], px);
      pw = fma(a[rr][u], wvv[u], pw);
      if (want_sq) sq = fma(a[rr][u], a[rr][u], sq);
    }
    v[rr] = px;
    v[RC + rr] = pw;
  }
  const double s = wave_multi_sum<NV>(v, lane);
  if ((lane & ((1 << SH) - 1)) == 0) sred[wv][lane >> SH] = s;
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < RC; ++rr) {
    const double y = ((sred[0][rr] + sred[1][rr]) + sred[2][rr]) + sred[3][rr];
    const double yw = ((sred[0][RC + rr] + sred[1][RC + rr]) + sred[2][RC + rr]) + sred[3][RC + rr];
#pragma unroll
    for (int u = 0; u < NC; ++u) z[u] = fma(a[rr][u], y, z[u]);
    ex = fma(y, y, ex);
    ew = fma(yw, yw, ew);
  }
}

template <typename TA, int LY, int NC>
__global__ __launch_bounds__(kPT) void k_defl_pass(const TA* __restrict__ A, int64_t m, int n,
                                                   const double* __restrict__ x, const double* __restrict__ w,
                                                   int want_sq, int64_t band, double* __restrict__ part) {
  constexpr int RC = NC >= kPerThread ? 1 : kPerThread / NC;   // rows per chunk
  constexpr int NV = 2 * RC;                                    // row products per chunk: A x and A w
  // two buffers: a chunk's writes never meet the previous chunk's reads, so one
  // barrier per chunk orders them (a thread passes chunk k + 1's barrier only
  // after its own reads of chunk k)
  __shared__ double sred[2][kPT / 64][NV];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const bool hx = x != nullptr, hw = w != nullptr;
  double xv[NC], wvv[NC], z[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int col = t + kPT * u;
    xv[u] = (hx && col < n) ? x[col] : 0.0;
    wvv[u] = (hw && col < n) ? w[col] : 0.0;
    z[u] = 0.0;
  }
  double ex = 0.0, ew = 0.0, sq = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * band;
  const int64_t r1 = (r0 + band < m) ? r0 + band : m;
  // one chunk at a time: the workgroups resident on a CU keep each other's
  // loads in flight
  int buf = 0;
  int64_t i0 = r0;
  for (; i0 + RC <= r1; i0 += RC) {
    double a[RC][NC];
    pass_load<true, TA, LY, NC, RC>(A, m, n, i0, r1, a);
    pass_chunk<NC, RC>(a, xv, wvv, z, ex, ew, sq, want_sq, sred[buf]);
    buf ^= 1;
  }
  if (i0 < r1) {
    double a[RC][NC];
    pass_load<false, TA, LY, NC, RC>(A, m, n, i0, r1, a);
    pass_chunk<NC, RC>(a, xv, wvv, z, ex, ew, sq, want_sq, sred[buf]);
  }
  double* out = part + (int64_t)blockIdx.x * (n + 3);
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int col = t + kPT * u;
    if (col < n) out[col] = hx ? z[u] : 0.0;
  }
  // ||A||^2 over the band: wave sums, then the four in order
  for (int o = 32; o >= 1; o >>= 1) sq += __shfl_xor(sq, o, 64);
  __syncthreads();   // the last chunk's readers of sred are done
  if (lane == 0) sred[0][wv][0] = sq;
  __syncthreads();
  if (t == 0) {
    out[n] = ex;
    out[n + 1] = ew;
    out[n + 2] = ((sred[0][0][0] + sred[0][1][0]) + sred[0][2][0]) + sred[0][3][0];
  }
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// The same pass with one wave per workgroup, for n <= 512 on row-major A and
// n <= 128 on column-major A (lane l keeps the columns l + 64 u, u < NC): a
// chunk's row products are summed by the wave's halving butterfly alone and
// read back with v_readlane, so no barrier and no LDS; many small workgroups
// keep the CUs' load queues full.  (Column-major A with wide n would leave each
// lane reading 16-byte runs of one column.)
template <typename TA, int LY, int NC>
__global__ __launch_bounds__(64) void k_defl_pass_w(const TA* __restrict__ A, int64_t m, int n,
                                                    const double* __restrict__ x, const double* __restrict__ w,
                                                    int want_sq, int64_t band, double* __restrict__ part) {
  constexpr int RC = NC >= kPerThread ? 1 : kPerThread / NC;
  constexpr int NV = 2 * RC;
  constexpr int SH = 6 - log2c<NV>();
  const int lane = threadIdx.x;
  const bool hx = x != nullptr, hw = w != nullptr;
  double xv[NC], wvv[NC], z[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int col = lane + 64 * u;
    xv[u] = (hx && col < n) ? x[col] : 0.0;
    wvv[u] = (hw && col < n) ? w[col] : 0.0;
    z[u] = 0.0;
  }
  double ex = 0.0, ew = 0.0, sq = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * band;
  const int64_t r1 = (r0 + band < m) ? r0 + band : m;
  auto chunk = [&](const double (&a)[RC][NC]) {
    double v[NV];
#pragma unroll
    for (int rr = 0; rr < RC; ++rr) {
      double px = 0.0, pw = 0.0;
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        px = fma(a[rr][u], xv[u], px);
        pw = fma(a[rr][u], wvv[u], pw);
        if (want_sq) sq = fma(a[rr][u], a[rr][u], sq);
      }
      v[rr] = px;
      v[RC + rr] = pw;
    }
    const double s = wave_multi_sum<NV>(v, lane);
#pragma unroll
    for (int rr = 0; rr < RC; ++rr) {
      const double y = readlane_d(s, rr << SH);
      const double yw = readlane_d(s, (RC + rr) << SH);
#pragma unroll
      for (int u = 0; u < NC; ++u) z[u] = fma(a[rr][u], y, z[u]);
      ex = fma(y, y, ex);
      ew = fma(yw, yw, ew);
    }
  };
  int64_t i0 = r0;
  for (; i0 + RC <= r1; i0 += RC) {
    double a[RC][NC];
#pragma unroll
    for (int rr = 0; rr < RC; ++rr) {
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const int64_t i = i0 + rr;
        const int col = lane + 64 * u;
        const int cc = col < n ? col : n - 1;
        const double v = (double)A[LY == COL ? i + (int64_t)cc * m : i * n + cc];
        a[rr][u] = col < n ? v : 0.0;
      }
    }
    chunk(a);
  }
  if (i0 < r1) {
    double a[RC][NC];
#pragma unroll
    for (int rr = 0; rr < RC; ++rr) {
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const int64_t i = i0 + rr;
        const int col = lane + 64 * u;
        const int cc = col < n ? col : n - 1;
        a[rr][u] = (i < r1 && col < n) ? (double)A[LY == COL ? i + (int64_t)cc * m : i * n + cc] : 0.0;
      }
    }
    chunk(a);
  }
  double* out = part + (int64_t)blockIdx.x * (n + 3);
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int col = lane + 64 * u;
    if (col < n) out[col] = hx ? z[u] : 0.0;
  }
  for (int o = 32; o >= 1; o >>= 1) sq += __shfl_xor(sq, o, 64);
  if (lane == 0) {
    out[n] = ex;
    out[n + 1] = ew;
    out[n + 2] = sq;
  }
}

bool one_wave(int n, int layout) { return n <= (layout == COL ? kWaveMaxNCol : kWaveMaxN); }

template <typename TA, int LY>
hipError_t pass_nc(const TA* A, int64_t m, int n, const double* x, const double* w, int want_sq, double* part,
                   int groups, int64_t band, hipStream_t st) {
  const dim3 g((unsigned)groups), b(kPT), bw(64);
  if (one_wave(n, LY)) {
    if (n <= 64) TT_LAUNCH((k_defl_pass_w<TA, LY, 1>), g, bw, 0, st, A, m, n, x, w, want_sq, band, part);
    else if (n <= 128) TT_LAUNCH((k_defl_pass_w<TA, LY, 2>), g, bw, 0, st, A, m, n, x, w, want_sq, band, part);
    else if (n <= 256) TT_LAUNCH((k_defl_pass_w<TA, LY, 4>), g, bw, 0, st, A, m, n, x, w, want_sq, band, part);
    else TT_LAUNCH((k_defl_pass_w<TA, LY, 8>), g, bw, 0, st, A, m, n, x, w, want_sq, band, part);
    return hipGetLastError();
  }
  if (n <= kPT) TT_LAUNCH((k_defl_pass<TA, LY, 1>), g, b, 0, st, A, m, n, x, w, want_sq, band, part);
  else if (n <= 2 * kPT) TT_LAUNCH((k_defl_pass<TA, LY, 2>), g, b, 0, st, A, m, n, x, w, want_sq, band, part);
  else if (n <= 4 * kPT) TT_LAUNCH((k_defl_pass<TA, LY, 4>), g, b, 0, st, A, m, n, x, w, want_sq, band, part);
  else if (n <= 8 * kPT) TT_LAUNCH((k_defl_pass<TA, LY, 8>), g, b, 0, st, A, m, n, x, w, want_sq, band, part);
  else TT_LAUNCH((k_defl_pass<TA, LY, 16>), g, b, 0, st, A, m, n, x, w, want_sq, band, part);
  return hipGetLastError();
}

int64_t pass_band(int64_t m, int groups) {
  const int64_t b = (m + groups - 1) / groups;
  return b < 1 ? 1 : b;
}

}  // namespace

int defl_pass_groups(int64_t m, int n, int layout) {
  // one-wave workgroups: at least 16 rows each, up to 8192 (measured on a
  // 4,096,000 x 160 row-major pass: 989 us at 8192 against 1141 us at 4096);
  // four-wave workgroups: at least 64 rows each, up to 1024, and on a short A
  // at least 16 rows each, up to 64
  const bool wave = one_wave(n, layout);
  int64_t g = wave ? (m + 15) / 16 : (m + 63) / 64;
  const int64_t cap = wave ? 8192 : 1024;
  if (g > cap) g = cap;
  if (!wave && g < 64) {   // a short, wide A: bands of 16 rows, up to 64 workgroups
    const int64_t g16 = (m + 15) / 16;
    g = g16 < 64 ? g16 : 64;
  }
  return g < 1 ? 1 : (int)g;
}

int64_t defl_pass_scratch(int64_t m, int n_max, int layout) {
  // the pass partials for any core side n <= n_max (a prescribed-accuracy step
  // learns its n at run time; the one-wave form, taken below a width threshold,
  // has the most workgroups), plus the stripes of their two-stage reduction
  const int thr = layout == COL ? kWaveMaxNCol : kWaveMaxN;
  int64_t most = 0;
  const int nw = n_max < thr ? n_max : thr;
  if (nw >= 1) most = (int64_t)defl_pass_groups(m, nw, layout) * (nw + 3);
  if (n_max > thr) {
    const int64_t g4 = (int64_t)defl_pass_groups(m, n_max, layout) * (n_max + 3);
    if (g4 > most) most = g4;
  }
  return most + (int64_t)kReduceStripes * (n_max + 3);
}

hipError_t launch_defl_pass(const void* A, int a_f32, int64_t m, int n, int layout, const double* x,
                            const double* w, int want_sq, double* part, int groups, hipStream_t st) {
  if (!A || m < 1 || n < 1 || n > kDeflMaxN || groups < 1 || !part) return hipErrorInvalidValue;
  const int64_t band = pass_band(m, groups);   // trailing bands may be empty: they write zero partials
  if (a_f32) {
    if (layout == COL) return pass_nc<float, COL>((const float*)A, m, n, x, w, want_sq, part, groups, band, st);
    return pass_nc<float, ROW>((const float*)A, m, n, x, w, want_sq, part, groups, band, st);
  }
  if (layout == COL) return pass_nc<double, COL>((const double*)A, m, n, x, w, want_sq, part, groups, band, st);
  return pass_nc<double, ROW>((const double*)A, m, n, x, w, want_sq, part, groups, band, st);
}

}  // namespace ttutv
