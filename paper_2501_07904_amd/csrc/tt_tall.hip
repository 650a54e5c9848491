// Streaming kernels over the tall side of an unfolding: the passes that read
// the m x n matrix A from HBM.  All accumulation is FP64; partial sums per row
// chunk are reduced in a fixed order, so results are bitwise reproducible.
#include <type_traits>

#include "tt_internal.h"

namespace ttutv {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t at(int layout, int64_t i, int64_t j, int64_t m, int64_t n) {
  return layout == ROW ? i * n + j : i + j * m;
}

template <typename T>
__device__ __forceinline__ double ldv(const T* p, int64_t i) { return (double)p[i]; }

__device__ __forceinline__ double group_sum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

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
// Row tiles and column blocks that fix the chunking of the A^T Y passes
// (atb_chunks): 32-row tiles, 64-column blocks.
constexpr int kAtbTR = 32;
constexpr int kAtbJT = 64;

// ---------------------------------------------------------------------------
// Y = A W on the FP64 matrix cores.  W (n x c) is k-major (row k = c
// contiguous doubles).  A workgroup (4 waves) owns a 64-row tile; wave w owns
// rows 16w..16w+15 and computes the 16 x 16*NT block of Y with
// v_mfma_f64_16x16x4 (operand A: lane l holds row l%16 at k-slot l/16;
// operand B: lane l holds column l%16 at k-slot l/16; result: lane l,
// register v holds row l/16 + 4v, column l%16).  The k-slots are mapped to
// contiguous k: in a 32-wide k block, lanes of group g = l/16 take
// k = 8g .. 8g+7 over eight consecutive MFMAs, so every lane streams eight
// consecutive elements of its row (ROW layout) and every group of 16 lanes
// reads 16 consecutive rows (COL layout).  W is staged 64 k at a time in LDS.
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kAxKC = 64;
constexpr int kAxSplitTiles = 128;   // A*W splits its k range when A has fewer 64-row tiles

// Loads of one KC-column chunk of A for the MFMA operand of this lane:
// a[ss*8 + s8] = A(row, k0 + 32 ss + 8 g + s8), zero outside the matrix.
template <typename TA, int LY, int KC>
__device__ __forceinline__ void ax_load_chunk(const TA* __restrict__ A, int64_t m, int n, int64_t row, bool rok,
                                              int k0, int k_end, double* a) {
  const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int ss = 0; ss < KC / 32; ++ss) {
    const int kb = k0 + 32 * ss + 8 * g;
    const TA* p = (LY == ROW) ? A + row * n + kb : A + row + (int64_t)kb * m;
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) {
      const bool ok = rok && kb + s8 < k_end;
      a[ss * 8 + s8] = ok ? (double)p[(LY == ROW) ? (int64_t)s8 : (int64_t)s8 * m] : 0.0;
    }
  }
}

// Accumulate the 64-row tile `tile` of Y = A W over columns [k_begin, k_end)
// of A into acc; ssa collects the sum of squares of the A entries read.  The
// chunk loop is software-pipelined: the loads of chunk k+1 of A (registers)
// and of W (into the other half of the double-buffered sW) are in flight
// while chunk k runs on the matrix cores; one barrier per chunk.  KC = 32
// for the wider W operands (NT >= 3) and for column-major A (one address per
// loaded column) keeps the two A buffers, the W staging and the accumulators
// in registers.
template <typename TA, int NT, int LY, int KC>
__device__ __forceinline__ void ax_accumulate(const TA* __restrict__ A, const double* __restrict__ W,
                                              double (*sW)[KC][NT * 16 + 1], int64_t m, int n, int c,
                                              int64_t tile, int k_begin, int k_end, d4* acc, double& ssa) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t row = tile * 64 + 16 * w + li;
  const bool rok = row < m;
  constexpr int NA = KC / 4;   // A values per lane per chunk
  constexpr int NWS = (KC * NT * 16 + kThreads - 1) / kThreads;
  if (k_begin >= k_end) return;
  double a[NA], an[NA], wn[NWS];
  auto load_w = [&](int k0, double* dst) {
    const int kc = min(KC, k_end - k0);
#pragma unroll
    for (int u = 0; u < NWS; ++u) {
      const int e = threadIdx.x + kThreads * u;
      const int kk = e / (NT * 16), cc = e % (NT * 16);
      dst[u] = (e < KC * NT * 16 && kk < kc && cc < c) ? W[(int64_t)(k0 + kk) * c + cc] : 0.0;
    }
  };
  auto store_w = [&](const double* src, int buf) {
#pragma unroll
    for (int u = 0; u < NWS; ++u) {
      const int e = threadIdx.x + kThreads * u;
      if (e < KC * NT * 16) sW[buf][e / (NT * 16)][e % (NT * 16)] = src[u];
    }
  };
  __syncthreads();   // sW may still be read by a previous tile
  load_w(k_begin, wn);
  ax_load_chunk<TA, LY, KC>(A, m, n, row, rok, k_begin, k_end, a);
  store_w(wn, 0);
  __syncthreads();
  int buf = 0;
  for (int k0 = k_begin; k0 < k_end; k0 += KC) {
    const int k1 = k0 + KC;
    const bool more = k1 < k_end;
    if (more) {
      load_w(k1, wn);
      ax_load_chunk<TA, LY, KC>(A, m, n, row, rok, k1, k_end, an);
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) ssa = fma(a[u], a[u], ssa);
#pragma unroll
    for (int ss = 0; ss < KC / 32; ++ss) {
      const int kb = 32 * ss + 8 * g;
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma_f64(a[ss * 8 + s8], sW[buf][kb + s8][16 * t + li], acc[t]);
    }
    if (more) {
      store_w(wn, buf ^ 1);
#pragma unroll
      for (int u = 0; u < NA; ++u) a[u] = an[u];
    }
    __syncthreads();
    buf ^= 1;
  }
}

template <typename TA, typename TY, int NT, int LY>
__global__ __launch_bounds__(kThreads, 2) void k_ax(const TA* __restrict__ A, const double* __restrict__ W,
                                                 TY* __restrict__ Y, int64_t m, int n, int c,
                                                 double* __restrict__ sumsqA,
                                                 double* __restrict__ sumsqY, double* __restrict__ rerr) {
  constexpr int KC = (NT >= 3 || LY == COL) ? 32 : kAxKC;
  __shared__ double sW[2][KC][NT * 16 + 1];
  __shared__ double sh[8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  double ssa = 0.0, ssy = 0.0, sse = 0.0;
  for (int64_t tile = blockIdx.x; tile * 64 < m; tile += gridDim.x) {
    d4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    ax_accumulate<TA, NT, LY, KC>(A, W, sW, m, n, c, tile, 0, n, acc, ssa);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t yr = tile * 64 + 16 * w + g + 4 * v;
        const int col = 16 * t + li;
        if (yr < m && col < c) {
          const TY y = (TY)acc[t][v];
          const double yd = (double)y;
          ssy = fma(yd, yd, ssy);
          const double e = acc[t][v] - yd;
          sse = fma(e, e, sse);
          Y[at(LY, yr, col, m, c)] = y;
        }
      }
    }
  }
  if (sumsqA) {
    const double s = block_sum(ssa, sh);
    if (threadIdx.x == 0) sumsqA[blockIdx.x] = s;
  }
  if (sumsqY) {
    const double s = block_sum(ssy, sh);
    if (threadIdx.x == 0) sumsqY[blockIdx.x] = s;
  }
  if (rerr) {
    const double s = block_sum(sse, sh);
    if (threadIdx.x == 0) rerr[blockIdx.x] = s;
  }
}

// Short A (few row tiles): workgroup b owns rows 16b .. 16b+15; its 16 waves
// split the k range in slices of 32 columns (wave w takes slices w, w+16, ...).
// A wave issues all loads of a slice at once -- its 8 values of A and the
// matching 8*NT values of W, read straight from L2 into the MFMA operand
// registers -- then multiplies; the 16 partial 16 x 16*NT blocks are summed in
// LDS in wave order, so the result is independent of timing.
constexpr int kAxKwSlice = 32;
// 16 waves, or 8 when the wider W operand (NT >= 3) needs more registers per lane
__host__ __device__ constexpr int ax_kw_threads(int nt) { return nt <= 2 ? 1024 : 512; }

template <typename TA, typename TY, int NT, int LY>
__global__ __launch_bounds__(ax_kw_threads(NT)) void k_ax_kw(const TA* __restrict__ A, const double* __restrict__ W,
                                                        TY* __restrict__ Y, int64_t m, int n, int c,
                                                        double* __restrict__ sumsqA, double* __restrict__ sumsqY,
                                                        double* __restrict__ rerr) {
  constexpr int NTH = ax_kw_threads(NT);
  constexpr int NW = NTH / 64;
  __shared__ double sR[NW][16][NT * 16 + 1];
  __shared__ double sh[NW];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t row = (int64_t)blockIdx.x * 16 + li;
  const bool rok = row < m;
  const int nslices = (n + kAxKwSlice - 1) / kAxKwSlice;
  double ssa = 0.0;
  d4 acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  for (int sl = w; sl < nslices; sl += NW) {
    const int kb = sl * kAxKwSlice + 8 * g;   // k of this lane's k-slot at step s8: kb + s8
    double a[8], b[8][NT];
    const TA* p = (LY == ROW) ? A + row * n + kb : A + row + (int64_t)kb * m;
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) {
      const int k = kb + s8;
      a[s8] = (rok && k < n) ? (double)p[(LY == ROW) ? (int64_t)s8 : (int64_t)s8 * m] : 0.0;
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int col = 16 * q + li;
        b[s8][q] = (k < n && col < c) ? W[(int64_t)k * c + col] : 0.0;
      }
    }
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) {
      ssa = fma(a[s8], a[s8], ssa);
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[q] = mfma_f64(a[s8], b[s8][q], acc[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) sR[w][g + 4 * v][16 * q + li] = acc[q][v];
  __syncthreads();
  double ssy = 0.0, sse = 0.0;
  for (int e = t; e < 16 * c; e += NTH) {
    int rr, col;
    if (LY == ROW) { rr = e / c; col = e % c; } else { rr = e % 16; col = e / 16; }
    const int64_t yr = (int64_t)blockIdx.x * 16 + rr;
    if (yr >= m) continue;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) sum += sR[q][rr][col];
    const TY y = (TY)sum;
    const double yd = (double)y;
    ssy = fma(yd, yd, ssy);
    const double er = sum - yd;
    sse = fma(er, er, sse);
    Y[at(LY, yr, col, m, c)] = y;
  }
  // block sums (fixed order over the waves)
  auto bsum = [&](double v) {
    v = group_sum64(v);
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s2 = 0.0;
    for (int q = 0; q < NW; ++q) s2 += sh[q];
    return s2;
  };
  if (sumsqA) {
    const double s2 = bsum(ssa);
    if (t == 0) sumsqA[blockIdx.x] = s2;
  }
  if (sumsqY) {
    const double s2 = bsum(ssy);
    if (t == 0) sumsqY[blockIdx.x] = s2;
  }
  if (rerr) {
    const double s2 = bsum(sse);
    if (t == 0) rerr[blockIdx.x] = s2;
  }
}

// ---------------------------------------------------------------------------
// Narrow A (n <= 64 columns).  No LDS staging and no block barrier in the row
// loop: every wave streams its own 16-row blocks straight into the MFMA
// operands, prefetching the next block while the current one is multiplied.
// Within a block of 16 rows the k-slot g of MFMA step s is row 4s + g, so one
// load instruction covers four consecutive rows of 16 columns.

// partials[chunk] = A^T A over the rows of chunk (n <= 64, NB = ceil(n/16)
// column blocks).  Only the blocks I <= J are multiplied (both operands of a
// Gram block come from the same registers); the lower blocks are written by
// symmetry.  The four waves' partial blocks are summed in LDS in wave order.
// Each lane takes a run of RPL consecutive rows (RPL = 64 bytes of each
// column: 16 FP32 or 8 FP64 values) as vector loads when the storage is
// column-major and aligned (VEC), so that a wave's loads cover 4 x 64
// contiguous bytes of each of 16 columns; MFMA step s then uses row RPL g + s
// for k-slot g, and a wave advances 4 RPL rows per iteration.
template <typename TA, int NB, int LY, bool VEC>
__global__ __launch_bounds__(kThreads) void k_gram_narrow(const TA* __restrict__ A, int64_t m, int n,
                                                          int64_t rows_per_chunk, double* __restrict__ partials) {
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr int RPL = 64 / (int)sizeof(TA);
  constexpr int RW = 4 * RPL;   // rows per wave iteration
  __shared__ double sR[kThreads / 64][NP][16][17];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(m, r0 + rows_per_chunk);
  d4 acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  typedef TA vec_t __attribute__((ext_vector_type(4)));
  auto load = [&](int64_t i0, TA (*a)[RPL]) {
    const int64_t ib = i0 + RPL * g;   // first row of this lane's run
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = 16 * b + li;
      const bool jok = j < n;
      if (VEC && LY == COL) {
        const TA* p = A + ib + (int64_t)j * m;
        if (jok && ib + RPL <= r1) {
#pragma unroll
          for (int h = 0; h < RPL / 4; ++h) {
            const vec_t v = *reinterpret_cast<const vec_t*>(p + 4 * h);
#pragma unroll
            for (int e = 0; e < 4; ++e) a[b][4 * h + e] = v[e];
          }
        } else {
#pragma unroll
          for (int s4 = 0; s4 < RPL; ++s4) a[b][s4] = (jok && ib + s4 < r1) ? p[s4] : (TA)0;
        }
      } else {
#pragma unroll
        for (int s4 = 0; s4 < RPL; ++s4) {
          const int64_t i = ib + s4;
          a[b][s4] = (jok && i < r1) ? A[LY == ROW ? i * n + j : i + (int64_t)j * m] : (TA)0;
        }
      }
    }
  };
  TA a[NB][RPL], an[NB][RPL];
  int64_t i0 = r0 + RW * w;
  if (i0 < r1) load(i0, a);
  for (; i0 < r1; i0 += RW * (kThreads / 64)) {
    const int64_t i1 = i0 + RW * (kThreads / 64);
    if (i1 < r1) load(i1, an);
#pragma unroll
    for (int s4 = 0; s4 < RPL; ++s4) {
      int q = 0;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NB; ++bj, ++q) acc[q] = mfma_f64((double)a[bi][s4], (double)a[bj][s4], acc[q]);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int s4 = 0; s4 < RPL; ++s4) a[b][s4] = an[b][s4];
  }
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) sR[w][q][g + 4 * v][li] = acc[q][v];
  __syncthreads();
  double* out = partials + (int64_t)blockIdx.x * n * n;
  for (int e = t; e < NP * 256; e += kThreads) {
    const int q = e >> 8, rr = (e >> 4) & 15, cc = e & 15;
    int bi = 0, bj = 0, k = 0;
#pragma unroll
    for (int x = 0; x < NB; ++x)
#pragma unroll
      for (int y = x; y < NB; ++y, ++k)
        if (k == q) { bi = x; bj = y; }
    const double v = ((sR[0][q][rr][cc] + sR[1][q][rr][cc]) + (sR[2][q][rr][cc] + sR[3][q][rr][cc]));
    const int j = 16 * bi + rr, c2 = 16 * bj + cc;
    if (j < n && c2 < n) {
      out[j + (int64_t)n * c2] = v;
      if (bi != bj) out[c2 + (int64_t)n * j] = v;
    }
  }
}

// Y = A W for n <= 64: W (k-major) stays in registers as the B operand for the
// whole launch (lane (g, li) holds W(4s + g, 16t + li)); each wave streams
// 16-row blocks; the result block goes through a wave-private LDS tile so that
// Y is written in full cache lines (16 consecutive rows of a column, or the
// contiguous 16 x c block in row-major storage).
template <typename TA, typename TY, int NT, int NK, int LY>
__global__ __launch_bounds__(kThreads) void k_ax_narrow(const TA* __restrict__ A, const double* __restrict__ W,
                                                        TY* __restrict__ Y, int64_t m, int n, int c,
                                                        double* __restrict__ sumsqA, double* __restrict__ sumsqY,
                                                        double* __restrict__ rerr) {
  __shared__ double sT[kThreads / 64][16][NT * 16 + 1];
  __shared__ double sh[8];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  double wr[NK][NT];
#pragma unroll
  for (int s4 = 0; s4 < NK; ++s4)
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int k = 4 * s4 + g, col = 16 * q + li;
      wr[s4][q] = (k < n && col < c) ? W[(int64_t)k * c + col] : 0.0;
    }
  double ssa = 0.0, ssy = 0.0, sse = 0.0;
  const int64_t nblk = (m + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * (kThreads / 64);
  auto load = [&](int64_t b, double* a) {
    const int64_t row = b * 16 + li;
    const bool rok = row < m;
#pragma unroll
    for (int s4 = 0; s4 < NK; ++s4) {
      const int k = 4 * s4 + g;
      a[s4] = (rok && k < n) ? (double)A[LY == ROW ? row * n + k : row + (int64_t)k * m] : 0.0;
    }
  };
  double a[NK], an[NK];
  int64_t b = (int64_t)blockIdx.x * (kThreads / 64) + w;
  if (b < nblk) load(b, a);
  for (; b < nblk; b += stride) {
    if (b + stride < nblk) load(b + stride, an);
    d4 acc[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < NK; ++s4) {
      if (4 * s4 < n) {   // k-steps past the last column only add zeros (skipped, not broken out of:
                          // a break keeps the loop rolled and wr, a in scratch memory)
        ssa = fma(a[s4], a[s4], ssa);
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[q] = mfma_f64(a[s4], wr[s4][q], acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) sT[w][g + 4 * v][16 * q + li] = acc[q][v];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int e = lane; e < 16 * c; e += 64) {
      int rr, col;
      if (LY == ROW) { rr = e / c; col = e % c; } else { rr = e & 15; col = e >> 4; }
      const int64_t yr = b * 16 + rr;
      if (yr < m) {
        const double s = sT[w][rr][col];
        const TY y = (TY)s;
        const double yd = (double)y;
        ssy = fma(yd, yd, ssy);
        const double er = s - yd;
        sse = fma(er, er, sse);
        Y[at(LY, yr, col, m, c)] = y;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int s4 = 0; s4 < NK; ++s4) a[s4] = an[s4];
  }
  if (sumsqA) {
    const double s = block_sum(ssa, sh);
    if (t == 0) sumsqA[blockIdx.x] = s;
  }
  if (sumsqY) {
    const double s = block_sum(ssy, sh);
    if (t == 0) sumsqY[blockIdx.x] = s;
  }
  if (rerr) {
    const double s = block_sum(sse, sh);
    if (t == 0) rerr[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// BF16 power-iteration products of the mixed-precision form (FP32
// accumulation on v_mfma_f32_16x16x16_bf16: operand A lane l holds row l%16 at
// k = 4(l/16) .. 4(l/16)+3, operand B lane l holds column l%16 at the same k,
// result lane l register v holds row 4(l/16)+v, column l%16).  Inputs are
// rounded to BF16 (nearest even) as they are loaded.
typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (short)(u >> 16);   // inf / nan pass through
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ f4 mfma_bf16(bf4 a, bf4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Y (m x c, FP32, layout LY) = A W on FP32-accumulating matrix cores with the
// operands rounded to BF16 (BF) or kept FP32 (v_mfma_f32_16x16x4_f32: operand A
// lane l holds row l%16 at k = l/16, operand B column l%16 at k = l/16, result
// as for BF16).  Workgroup = 64-row tile, wave w rows 16w .. 16w+15, k in
// chunks of 64 with W staged in LDS column-wise.
// FP32-operand form of ax_accumulate (v_mfma_f32_16x16x4_f32, k-slot g of step
// u is column 4u + g): W double-buffered in LDS as FP32, the next chunk of A
// loaded while the current one is multiplied, one barrier per chunk.
template <typename TA, int NT, int LY>
__device__ __forceinline__ void ax_accumulate_f32(const TA* __restrict__ A, const double* __restrict__ W,
                                                  float (*sW)[kAxKC][NT * 16 + 1], int64_t m, int n, int c,
                                                  int64_t tile, f4* acc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t row = tile * 64 + 16 * w + li;
  const bool rok = row < m;
  constexpr int NA = kAxKC / 4;
  constexpr int NWS = (kAxKC * NT * 16 + kThreads - 1) / kThreads;
  float a[NA], an[NA], wn[NWS];
  auto load_a = [&](int k0, float* dst) {
    const TA* p = (LY == ROW) ? A + row * n + k0 + g : A + row + (int64_t)(k0 + g) * m;
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const bool ok = rok && k0 + 4 * u + g < n;
      dst[u] = ok ? (float)p[(LY == ROW) ? (int64_t)4 * u : (int64_t)4 * u * m] : 0.f;
    }
  };
  auto load_w = [&](int k0, float* dst) {
    const int kc = min(kAxKC, n - k0);
#pragma unroll
    for (int u = 0; u < NWS; ++u) {
      const int e = threadIdx.x + kThreads * u;
      const int kk = e / (NT * 16), cc = e % (NT * 16);
      dst[u] = (e < kAxKC * NT * 16 && kk < kc && cc < c) ? (float)W[(int64_t)(k0 + kk) * c + cc] : 0.f;
    }
  };
  auto store_w = [&](const float* src, int buf) {
#pragma unroll
    for (int u = 0; u < NWS; ++u) {
      const int e = threadIdx.x + kThreads * u;
      if (e < kAxKC * NT * 16) sW[buf][e / (NT * 16)][e % (NT * 16)] = src[u];
    }
  };
  __syncthreads();
  load_w(0, wn);
  load_a(0, a);
  store_w(wn, 0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < n; k0 += kAxKC) {
    const int k1 = k0 + kAxKC;
    const bool more = k1 < n;
    if (more) {
      load_w(k1, wn);
      load_a(k1, an);
    }
#pragma unroll
    for (int u = 0; u < NA; ++u)
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[q] = mfma_f32(a[u], sW[buf][4 * u + g][16 * q + li], acc[q]);
    if (more) {
      store_w(wn, buf ^ 1);
#pragma unroll
      for (int u = 0; u < NA; ++u) a[u] = an[u];
    }
    __syncthreads();
    buf ^= 1;
  }
}

template <typename TA, int NT, int LY>
__global__ __launch_bounds__(kThreads, 2) void k_ax_f32(const TA* __restrict__ A, const double* __restrict__ W,
                                                        float* __restrict__ Y, int64_t m, int n, int c) {
  __shared__ float sW[2][kAxKC][NT * 16 + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  for (int64_t tile = blockIdx.x; tile * 64 < m; tile += gridDim.x) {
    f4 acc[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    ax_accumulate_f32<TA, NT, LY>(A, W, sW, m, n, c, tile, acc);
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t yr = tile * 64 + 16 * w + 4 * g + v;
        const int col = 16 * q + li;
        if (yr < m && col < c) Y[at(LY, yr, col, m, c)] = acc[q][v];
      }
  }
}

template <typename TA, int NT, int LY, bool BF>
__global__ __launch_bounds__(kThreads) void k_ax_lp(const TA* __restrict__ A, const double* __restrict__ W,
                                                    float* __restrict__ Y, int64_t m, int n, int c) {
  __shared__ __align__(16) short sWb[BF ? NT * 16 : 1][kAxKC + 4];
  __shared__ float sWf[BF ? 1 : NT * 16][kAxKC + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  for (int64_t tile = blockIdx.x; tile * 64 < m; tile += gridDim.x) {
    const int64_t row = tile * 64 + 16 * w + li;
    const bool rok = row < m;
    f4 acc[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < n; k0 += kAxKC) {
      const int kc = min(kAxKC, n - k0);
      __syncthreads();
      for (int e = t; e < kAxKC * NT * 16; e += kThreads) {
        const int kk = e / (NT * 16), cc = e % (NT * 16);
        const float v = (kk < kc && cc < c) ? (float)W[(int64_t)(k0 + kk) * c + cc] : 0.f;
        if constexpr (BF) sWb[cc][kk] = bf16_rne(v);
        else sWf[cc][kk] = v;
      }
      __syncthreads();
      // k of value u of this lane: BF: 16(u/4) + 4g + u%4; FP32: 4u + g
      float av[kAxKC / 4];
#pragma unroll
      for (int u = 0; u < kAxKC / 4; ++u) {
        const int k = k0 + (BF ? 16 * (u >> 2) + 4 * g + (u & 3) : 4 * u + g);
        av[u] = (rok && k < n) ? (float)A[LY == ROW ? row * n + k : row + (int64_t)k * m] : 0.f;
      }
      if constexpr (BF) {
#pragma unroll
        for (int s4 = 0; s4 < kAxKC / 16; ++s4) {
          bf4 a;
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = bf16_rne(av[4 * s4 + i]);
#pragma unroll
          for (int q = 0; q < NT; ++q) {
            const bf4 b = *reinterpret_cast<const bf4*>(&sWb[16 * q + li][16 * s4 + 4 * g]);
            acc[q] = mfma_bf16(a, b, acc[q]);
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < kAxKC / 4; ++u)
#pragma unroll
          for (int q = 0; q < NT; ++q) acc[q] = mfma_f32(av[u], sWf[16 * q + li][4 * u + g], acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t yr = tile * 64 + 16 * w + 4 * g + v;
        const int col = 16 * q + li;
        if (yr < m && col < c) Y[at(LY, yr, col, m, c)] = acc[q][v];
      }
  }
}

// partials[chunk] = A[rows of chunk, j0:j0+64]^T Y[rows of chunk, :] on
// FP32-accumulating matrix cores, operands rounded to BF16 (BF) or kept FP32,
// stored as FP64.  Operands come straight from global memory: lane (g, li) of
// wave w takes column j0+16w+li of A and column 16q+li of Y at rows i0+4g ..
// i0+4g+3 (BF16, one MFMA per 16 rows) or at row i0+4s+g of step s (FP32,
// four MFMAs per 16 rows).
template <typename TA, int NT, int LY, bool BF>
__global__ __launch_bounds__(kThreads) void k_atb_lp(const TA* __restrict__ A, const float* __restrict__ Y,
                                                     int64_t m, int n, int c, int64_t rows_per_chunk,
                                                     double* __restrict__ partials) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t chunk = blockIdx.x;
  const int j0 = blockIdx.y * kAtbJT;
  const int j = j0 + 16 * w + li;
  const bool jok = j < n;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = min(m, r0 + rows_per_chunk);
  f4 acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
  if (j0 + 16 * w < n) {
    for (int64_t i0 = r0; i0 < r1; i0 += 16) {
      float av[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = BF ? i0 + 4 * g + i : i0 + 4 * i + g;
        av[i] = (jok && r < r1) ? (float)A[LY == ROW ? r * n + j : r + (int64_t)j * m] : 0.f;
      }
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int col = 16 * q + li;
        float bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t r = BF ? i0 + 4 * g + i : i0 + 4 * i + g;
          bv[i] = (col < c && r < r1) ? Y[LY == ROW ? r * c + col : r + (int64_t)col * m] : 0.f;
        }
        if constexpr (BF) {
          bf4 a, b;
#pragma unroll
          for (int i = 0; i < 4; ++i) { a[i] = bf16_rne(av[i]); b[i] = bf16_rne(bv[i]); }
          acc[q] = mfma_bf16(a, b, acc[q]);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[q] = mfma_f32(av[i], bv[i], acc[q]);
        }
      }
    }
  }
  double* out = partials + chunk * (int64_t)n * c;
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int jj = j0 + 16 * w + 4 * g + v, cc = 16 * q + li;
      if (jj < n && cc < c) out[jj + (int64_t)n * cc] = (double)acc[q][v];
    }
}

// ---------------------------------------------------------------------------
// partials[chunk] = A[rows of chunk, j0:j0+128]^T Y[rows of chunk, :] on the
// matrix cores: FP64 (v_mfma_f64_16x16x4, result lane l register v at row
// l/16 + 4v) or FP32 (v_mfma_f32_16x16x4_f32, row 4(l/16) + v); both take
// operand A as lane l -> (row l%16, k l/16) and operand B as (k l/16, column
// l%16), the k-slots running over the rows of the tile.  Eight waves own 16
// columns of A each, so one staged tile of Y serves 128 columns.  Row tiles
// (32 rows) of A and Y are loaded with coalesced reads into registers one
// tile ahead (the loads of tile t+1 are in flight while tile t is
// multiplied), then stored to LDS behind a barrier.  VEC (column-major,
// aligned A, chunks of whole tiles): each lane reads 16 contiguous bytes of
// one column of A per load (2 FP64 or 4 FP32 rows), at clamped in-range
// addresses with rows and columns outside the chunk zeroed when staged.
// The (chunk, column block) pairs are numbered chunk-major and dealt to the
// eight XCDs in contiguous runs (hardware workgroup b runs on XCD b % 8), so
// that the column blocks sharing a chunk's rows of Y mostly run on one XCD
// and read those rows once from HBM into its L2: dealt round-robin, each
// chunk's ten column blocks (n = 1280) spread over all eight XCDs and Y was
// fetched about eight times.
constexpr int kAtb2Threads = 512;
constexpr int kAtb2JB = 128;
constexpr int kAtb2TR = 32;

template <typename TA, typename TY, int NT, int LY, bool F32, bool VEC>
__global__ __launch_bounds__(kAtb2Threads) void k_atb2(const TA* __restrict__ A, const TY* __restrict__ Y, int64_t m,
                                                       int n, int c, int64_t rows_per_chunk, int nchunks,
                                                       double* __restrict__ partials) {
  typedef typename std::conditional<F32, float, double>::type T;
  typedef typename std::conditional<F32, f4, d4>::type V4;
  constexpr int NTH = kAtb2Threads;
  constexpr int WY = NT * 16;
  constexpr int LA = kAtb2TR * kAtb2JB / NTH;   // A values per thread per tile
  constexpr int VL = VEC ? 16 / (int)sizeof(TA) : 1;   // rows per vector load
  constexpr int LAV = LA / VL;                   // vector loads per thread per tile
  constexpr int LYV = (kAtb2TR * WY + NTH - 1) / NTH;
  typedef TA avec_t __attribute__((ext_vector_type(VL)));
  __shared__ T sA[kAtb2TR][kAtb2JB + 1];
  __shared__ T sY[kAtb2TR][WY + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int ncb = (n + kAtb2JB - 1) / kAtb2JB;
  const int64_t npairs = (int64_t)nchunks * ncb;
  const int64_t per_xcd = gridDim.x / 8;                // gridDim.x = roundup(npairs, 8)
  const int64_t pair = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (pair >= npairs) return;
  const int64_t chunk = pair / ncb;
  const int j0 = (int)(pair % ncb) * kAtb2JB;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = min(m, r0 + rows_per_chunk);
  // element e of a tile: COL -> (row e % TR, col e / TR); ROW -> (row e / W, col e % W);
  // VEC: vector e -> rows VL (e % (TR / VL)) .. + VL - 1 of col e / (TR / VL)
  T ra[LA], ry[LYV];
  avec_t rv[VEC ? LAV : 1];
  int64_t rb_cur = r0;   // first row of the tile whose loads are in flight
  auto load = [&](int64_t rb) {
    rb_cur = rb;
    if constexpr (VEC) {
#pragma unroll
      for (int u = 0; u < LAV; ++u) {
        const int e = t + NTH * u;
        const int i = (e % (kAtb2TR / VL)) * VL, j = e / (kAtb2TR / VL);
        int64_t r = rb + i;
        r = r < r1 - VL ? r : r1 - VL;                 // r1 - r0 is a multiple of VL
        const int jc = j0 + j < n ? j0 + j : n - 1;
        rv[u] = *reinterpret_cast<const avec_t*>(A + r + (int64_t)jc * m);
      }
    } else {
#pragma unroll
      for (int u = 0; u < LA; ++u) {
        const int e = t + NTH * u;
        int i, j;
        if (LY == ROW) { i = e / kAtb2JB; j = e % kAtb2JB; } else { i = e % kAtb2TR; j = e / kAtb2TR; }
        const int64_t r = rb + i;
        ra[u] = (r < r1 && j0 + j < n) ? (T)A[at(LY, r, j0 + j, m, n)] : (T)0;
      }
    }
#pragma unroll
    for (int u = 0; u < LYV; ++u) {
      const int e = t + NTH * u;
      int i, j;
      if (LY == ROW) { i = e / WY; j = e % WY; } else { i = e % kAtb2TR; j = e / kAtb2TR; }
      const int64_t r = rb + i;
      ry[u] = (e < kAtb2TR * WY && r < r1 && j < c) ? (T)Y[at(LY, r, j, m, c)] : (T)0;
    }
  };
  auto store = [&]() {
    if constexpr (VEC) {
#pragma unroll
      for (int u = 0; u < LAV; ++u) {
        const int e = t + NTH * u;
        const int i = (e % (kAtb2TR / VL)) * VL, j = e / (kAtb2TR / VL);
        const bool jok = j0 + j < n;
#pragma unroll
        for (int v = 0; v < VL; ++v) sA[i + v][j] = (jok && rb_cur + i + v < r1) ? (T)rv[u][v] : (T)0;
      }
    } else {
#pragma unroll
      for (int u = 0; u < LA; ++u) {
        const int e = t + NTH * u;
        int i, j;
        if (LY == ROW) { i = e / kAtb2JB; j = e % kAtb2JB; } else { i = e % kAtb2TR; j = e / kAtb2TR; }
        sA[i][j] = ra[u];
      }
    }
#pragma unroll
    for (int u = 0; u < LYV; ++u) {
      const int e = t + NTH * u;
      if (e >= kAtb2TR * WY) break;
      int i, j;
      if (LY == ROW) { i = e / WY; j = e % WY; } else { i = e % kAtb2TR; j = e / kAtb2TR; }
      sY[i][j] = ry[u];
    }
  };
  V4 acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = V4{0, 0, 0, 0};
  const bool active = j0 + 16 * w < n;
  if (r0 < r1) load(r0);
  for (int64_t rb = r0; rb < r1; rb += kAtb2TR) {
    __syncthreads();
    store();
    __syncthreads();
    if (rb + kAtb2TR < r1) load(rb + kAtb2TR);
    if (active) {
#pragma unroll
      for (int ks = 0; ks < kAtb2TR / 4; ++ks) {
        const int i = 4 * ks + g;
        const T a = sA[i][16 * w + li];
#pragma unroll
        for (int q = 0; q < NT; ++q) {
          if constexpr (F32) acc[q] = mfma_f32(a, sY[i][16 * q + li], acc[q]);
          else acc[q] = mfma_f64(a, sY[i][16 * q + li], acc[q]);
        }
      }
    }
  }
  double* out = partials + chunk * (int64_t)n * c;
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int jj = j0 + 16 * w + (F32 ? 4 * g + v : g + 4 * v), cc = 16 * q + li;
      if (jj < n && cc < c) out[jj + (int64_t)n * cc] = (double)acc[q][v];
    }
}

// ---------------------------------------------------------------------------
// One power product Z = A^T (A X) with each row tile of A read from HBM once
// (FP64, column-major A, n <= 512, n c <= 12288).  A workgroup of 8 waves
// walks 16-row tiles of its rows; wave w owns columns 64w .. 64w+63.
//   phase 1: Y_t = A_t X over the wave's columns (operand A: lane l holds
//            A(row l%16, column 64w + 4s + l/16) at k-step s; X, n x c
//            k-major, sits in LDS for the whole launch), the eight partial
//            16 x 16NT blocks summed in LDS in wave order (two barriers);
//   phase 2: Z(w's columns, :) += A_t^T Y_t (operand A: lane l holds
//            A(row 4s + l/16, column 64w + 16mt + l%16); the second reading
//            of the tile hits the caches), accumulated in registers.
// The next tile's phase-1 operand is loaded while the current one is
// multiplied.  Block b takes tiles b, b + B, b + 2B, ... (B blocks), so that
// at any moment the blocks read one contiguous band of rows of every column.
// Each workgroup writes its n x c partial of Z.
constexpr int kFaThreads = 512;
constexpr int kFaCW = 64;
constexpr int kFaTR = 16;
constexpr int kFaMaxN = 8 * kFaCW;
constexpr int kFaMaxNC = 12288;

template <int NT>
__global__ __launch_bounds__(kFaThreads) void k_fused_ata(const double* __restrict__ A, const double* __restrict__ X,
                                                          int64_t m, int n, int c,
                                                          double* __restrict__ partials) {
  constexpr int WY = 16 * NT;
  __shared__ double sX[kFaMaxNC];
  __shared__ double sP[8 * kFaTR * WY];
  __shared__ double sYt[kFaTR * WY];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int jw = kFaCW * w;
  const int64_t r0 = (int64_t)blockIdx.x * kFaTR, stride = (int64_t)gridDim.x * kFaTR;
  const int64_t r1 = m;
  for (int e = t; e < n * c; e += kFaThreads) sX[e] = X[e];
  double a1[16], a1n[16], a2[16];
  // loads stay straight-line: an index outside A is clamped into it and the
  // value replaced by zero afterwards
  auto load1 = [&](int64_t rb, double* dst) {
    const int64_t r = rb + li;
    const int64_t rc = r < r1 ? r : r1 - 1;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int j = jw + 4 * s + g;
      dst[s] = A[rc + m * (int64_t)(j < n ? j : n - 1)];
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int j = jw + 4 * s + g;
      dst[s] = (r < r1 && j < n) ? dst[s] : 0.0;
    }
  };
  auto load2 = [&](int64_t rb) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t r = rb + 4 * s + g;
        const int j = jw + 16 * mt + li;
        a2[4 * mt + s] = A[(r < r1 ? r : r1 - 1) + m * (int64_t)(j < n ? j : n - 1)];
      }
  };
  auto mask2 = [&](int64_t rb) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t r = rb + 4 * s + g;
        const int j = jw + 16 * mt + li;
        a2[4 * mt + s] = (r < r1 && j < n) ? a2[4 * mt + s] : 0.0;
      }
  };
  d4 z[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int q = 0; q < NT; ++q) z[mt][q] = d4{0, 0, 0, 0};
  if (r0 < r1) load1(r0, a1);
  __syncthreads();   // X staged
  for (int64_t rb = r0; rb < r1; rb += stride) {
    load2(rb);
    if (rb + stride < r1) load1(rb + stride, a1n);
    // phase 1
    d4 y[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) y[q] = d4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int j = jw + 4 * s + g;
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int col = 16 * q + li;
        const double xv = (j < n && col < c) ? sX[j * c + col] : 0.0;
        y[q] = mfma_f64(a1[s], xv, y[q]);
      }
    }
    // result lane l register v: row l/16 + 4v, column 16q + l%16
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) sP[(w * kFaTR + g + 4 * v) * WY + 16 * q + li] = y[q][v];
    __syncthreads();
    if (t < kFaTR * WY) {
      double sum = 0.0;
#pragma unroll
      for (int ww = 0; ww < 8; ++ww) sum += sP[ww * kFaTR * WY + t];
      sYt[t] = sum;
    }
    __syncthreads();
    // phase 2
    mask2(rb);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double yv[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) yv[q] = sYt[(4 * s + g) * WY + 16 * q + li];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int q = 0; q < NT; ++q) z[mt][q] = mfma_f64(a2[4 * mt + s], yv[q], z[mt][q]);
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) a1[s] = a1n[s];
  }
  double* out = partials + (int64_t)blockIdx.x * n * c;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = jw + 16 * mt + g + 4 * v, cc = 16 * q + li;
        if (jj < n && cc < c) out[jj + (int64_t)n * cc] = z[mt][q][v];
      }
}

// Column-major, aligned A (vector form of the narrow A*W): lane li of a wave
// owns the run of RB consecutive rows RB*li .. RB*li+RB-1 of a 16*RB-row block
// and loads it with one vector load per column; MFMA row block rb holds rows
// RB*li + rb.  W (n x c, at most 64 x 64) sits in LDS for the whole launch, so
// the waves run their blocks independently (no barrier after the set-up), each
// prefetching its next block while the current one runs on the matrix cores.
// Result row rho of block rb is block row RB*rho + rb: a lane holds RB
// consecutive rows of one column of Y and writes them with one vector store.
template <typename TA, typename TY, int NT, int NK, int RB>
__global__ __launch_bounds__(kThreads) void k_ax_narrow_v(const TA* __restrict__ A, const double* __restrict__ W,
                                                          TY* __restrict__ Y, int64_t m, int n, int c,
                                                          double* __restrict__ sumsqA, double* __restrict__ sumsqY,
                                                          double* __restrict__ rerr) {
  __shared__ double sW[4 * NK][NT * 16 + 1];
  __shared__ double sh[8];
  typedef TA vec_t __attribute__((ext_vector_type(RB)));
  typedef TY yvec_t __attribute__((ext_vector_type(RB)));
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  for (int e = t; e < 4 * NK * NT * 16; e += kThreads) {
    const int k = e / (NT * 16), col = e % (NT * 16);
    sW[k][col] = (k < n && col < c) ? W[(int64_t)k * c + col] : 0.0;
  }
  __syncthreads();
  double ssa = 0.0, ssy = 0.0, sse = 0.0;
  const int64_t nblk = (m + 16 * RB - 1) / (16 * RB);
  const int64_t stride = (int64_t)gridDim.x * (kThreads / 64);
  auto load = [&](int64_t b, vec_t* a) {
    const int64_t row = b * 16 * RB + RB * li;
    if (row + RB <= m) {
      const TA* p = A + row + (int64_t)g * m;
#pragma unroll
      for (int s4 = 0; s4 < NK; ++s4) {
        if (4 * s4 + g < n) a[s4] = *reinterpret_cast<const vec_t*>(p + (int64_t)(4 * s4) * m);
        else a[s4] = vec_t{};
      }
    } else {
#pragma unroll
      for (int s4 = 0; s4 < NK; ++s4) {
        const int k = 4 * s4 + g;
#pragma unroll
        for (int e = 0; e < RB; ++e) a[s4][e] = (k < n && row + e < m) ? A[row + e + (int64_t)k * m] : (TA)0;
      }
    }
  };
  vec_t a[NK], an[NK];
  int64_t b = (int64_t)blockIdx.x * (kThreads / 64) + w;
  if (b < nblk) load(b, a);
  for (; b < nblk; b += stride) {
    if (b + stride < nblk) load(b + stride, an);
    d4 acc[RB][NT];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[rb][q] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < NK; ++s4) {
      if (4 * s4 >= n) break;   // k-steps past the last column only add zeros
      double wv[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) wv[q] = sW[4 * s4 + g][16 * q + li];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const double x = (double)a[s4][rb];
        ssa = fma(x, x, ssa);
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[rb][q] = mfma_f64(x, wv[q], acc[rb][q]);
      }
    }
    // result register v holds MFMA row g + 4v, block row RB (g + 4v) + rb
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int col = 16 * q + li;
      if (col >= c) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r0 = b * 16 * RB + RB * (g + 4 * v);
        yvec_t yv;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const double sv = acc[rb][q][v];
          const TY y = (TY)sv;
          yv[rb] = y;
          if (r0 + rb < m) {
            const double yd = (double)y;
            ssy = fma(yd, yd, ssy);
            const double er = sv - yd;
            sse = fma(er, er, sse);
          }
        }
        if (r0 + RB <= m) {
          *reinterpret_cast<yvec_t*>(Y + r0 + (int64_t)col * m) = yv;
        } else {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            if (r0 + rb < m) Y[r0 + rb + (int64_t)col * m] = yv[rb];
        }
      }
    }
#pragma unroll
    for (int s4 = 0; s4 < NK; ++s4) a[s4] = an[s4];
  }
  if (sumsqA) {
    const double s = block_sum(ssa, sh);
    if (t == 0) sumsqA[blockIdx.x] = s;
  }
  if (sumsqY) {
    const double s = block_sum(ssy, sh);
    if (t == 0) sumsqY[blockIdx.x] = s;
  }
  if (rerr) {
    const double s = block_sum(sse, sh);
    if (t == 0) rerr[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Y = A W for column-major, aligned A of any width (vector form of k_ax).
// Lane li of a wave owns the run of RB consecutive rows RB*li .. RB*li+RB-1
// of the wave's 16*RB-row block and reads it with one vector load per column,
// so each load instruction covers 4 columns with 16*RB*sizeof(TA) contiguous
// bytes each; MFMA row block rb holds rows RB*li + rb.  The four waves own
// consecutive blocks (a 64*RB-row tile) and share each KC-column chunk of W,
// staged in LDS (double buffered).  The chunk loop is unrolled by two with
// two register buffers for A: the loads of chunk k+1 go to the other buffer
// while chunk k runs on the matrix cores.  Every load is issued
// unconditionally (clamped addresses, rows past m read row m-RB and columns
// past n read column n-1 of the same row): such values meet zero rows of W
// or land in rows that are never stored, and the sum of squares masks them.
// With no branch around a load and no copy between the buffers, the wait
// before a chunk's matrix-core block covers only that chunk's own loads (a
// conditional load or a register copy makes the compiler wait for the next
// chunk's loads there as well, which serialises memory and matrix cores).
// Result row rho of block rb is tile row RB*rho + rb, so a lane holds RB
// consecutive rows of one column of Y and writes them with one vector store.
// F32M: FP32 matrix cores (v_mfma_f32_16x16x4f32, A and W rounded to FP32,
// FP32 accumulation); otherwise FP64 matrix cores.  Requires m % RB == 0.
template <typename TA, typename TY, int NT, bool F32M, int RB, int KC>
__global__ __launch_bounds__(kThreads, 2) void k_ax_cv(const TA* __restrict__ A, const double* __restrict__ W,
                                                       TY* __restrict__ Y, int64_t m, int n, int c,
                                                       double* __restrict__ sumsqA, double* __restrict__ sumsqY,
                                                       double* __restrict__ rerr) {
  constexpr int TR = 4 * 16 * RB;            // rows per tile
  constexpr int NS = KC / 4;                 // k-steps per chunk
  constexpr int NWS = (KC * NT * 16 + kThreads - 1) / kThreads;
  typedef TA vec_t __attribute__((ext_vector_type(RB)));
  typedef TY yvec_t __attribute__((ext_vector_type(RB)));
  typedef typename std::conditional<F32M, float, double>::type TM;   // matrix-core operand type
  typedef typename std::conditional<F32M, f4, d4>::type acc_t;
  // FP32 rows padded by 4 words: the four k-rows a wave reads then fall on
  // distinct banks
  __shared__ TM sW[2][KC][NT * 16 + (sizeof(TM) == 4 ? 4 : 1)];
  __shared__ double sh[8];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  double ssa = 0.0, ssy = 0.0, sse = 0.0;
  const int64_t ntiles = (m + TR - 1) / TR;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * TR + 16 * RB * w + RB * li;   // first of this lane's RB rows
    const int64_t rowc = row < m - RB ? row : m - RB;
    auto load_a = [&](int k0, vec_t* a) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int k = k0 + 4 * s + g;
        const int kc = k < n ? k : n - 1;
        a[s] = *reinterpret_cast<const vec_t*>(A + rowc + (int64_t)kc * m);
      }
    };
    auto load_w = [&](int k0, TM* dst) {
#pragma unroll
      for (int u = 0; u < NWS; ++u) {
        const int e = t + kThreads * u;
        const int kk = e / (NT * 16), cc = e % (NT * 16);
        const bool ok = e < KC * NT * 16 && k0 + kk < n && cc < c;
        const double v = W[ok ? (int64_t)(k0 + kk) * c + cc : 0];
        dst[u] = ok ? (TM)v : (TM)0;
      }
    };
    auto store_w = [&](const TM* src, int buf) {
#pragma unroll
      for (int u = 0; u < NWS; ++u) {
        const int e = t + kThreads * u;
        if (e < KC * NT * 16) sW[buf][e / (NT * 16)][e % (NT * 16)] = src[u];
      }
    };
    acc_t acc[RB][NT];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[rb][q] = acc_t{0, 0, 0, 0};
    auto mma = [&](const vec_t* a, int buf, int k0) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        TM b[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) b[q] = sW[buf][4 * s + g][16 * q + li];
        const bool kok = k0 + 4 * s + g < n;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if constexpr (!F32M) {   // the FP32 form is launched without sums
            const double xd = (double)a[s][rb];
            ssa = fma(xd, (kok && row + rb < m) ? xd : 0.0, ssa);
          }
          const TM x = (TM)a[s][rb];
#pragma unroll
          for (int q = 0; q < NT; ++q) {
            if constexpr (F32M) acc[rb][q] = mfma_f32(x, b[q], acc[rb][q]);
            else acc[rb][q] = mfma_f64(x, b[q], acc[rb][q]);
          }
        }
      }
    };
    vec_t a0[NS], a1[NS];
    TM wn[NWS];
    __syncthreads();   // the previous tile's reads of sW are done
    load_w(0, wn);
    store_w(wn, 0);
    load_a(0, a0);
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += 2 * KC) {
      // chunk k0 in a0 / sW[0]; chunk k0 + KC in a1 / sW[1] (past the last
      // chunk: an unused clamped reload)
      const bool more1 = k0 + KC < n;
      load_w(k0 + KC, wn);
      load_a(more1 ? k0 + KC : k0, a1);
      mma(a0, 0, k0);
      store_w(wn, 1);
      __syncthreads();
      if (!more1) break;
      const bool more2 = k0 + 2 * KC < n;
      load_w(k0 + 2 * KC, wn);
      load_a(more2 ? k0 + 2 * KC : k0 + KC, a0);
      mma(a1, 1, k0 + KC);
      store_w(wn, 0);
      __syncthreads();
    }
    // result register v of a lane holds MFMA row rho = g + 4v (FP64) or 4g + v (FP32)
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int col = 16 * q + li;
      if (col >= c) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rho = F32M ? 4 * g + v : g + 4 * v;
        const int64_t r0 = tile * TR + 16 * RB * w + RB * rho;
        yvec_t yv;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const double s = (double)acc[rb][q][v];
          const TY y = (TY)s;
          yv[rb] = y;
          if (r0 + rb < m) {
            const double yd = (double)y;
            ssy = fma(yd, yd, ssy);
            const double er = s - yd;
            sse = fma(er, er, sse);
          }
        }
        if (r0 + RB <= m) {
          *reinterpret_cast<yvec_t*>(Y + r0 + (int64_t)col * m) = yv;
        } else {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            if (r0 + rb < m) Y[r0 + rb + (int64_t)col * m] = yv[rb];
        }
      }
    }
  }
  if (sumsqA) {
    const double s = block_sum(ssa, sh);
    if (t == 0) sumsqA[blockIdx.x] = s;
  }
  if (sumsqY) {
    const double s = block_sum(ssy, sh);
    if (t == 0) sumsqY[blockIdx.x] = s;
  }
  if (rerr) {
    const double s = block_sum(sse, sh);
    if (t == 0) rerr[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// resid[chunk] = sum over rows of ||A(i,:) - Cr(i,:) V1^T||^2 (direct step
// error); V1 (n x r) is stored k-major like the right operand of k_ax.
constexpr int kResTR = 64;
constexpr int kAxKT = 32;

template <typename TA, typename TC>
__global__ __launch_bounds__(kThreads) void k_resid(const TA* __restrict__ A, const TC* __restrict__ Cr,
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
      sC[i][a] = (double)Cr[at(layout, rb + i, a, m, r)];
    }
    for (int k0 = 0; k0 < n; k0 += kAxKT) {
      const int kt = min(kAxKT, n - k0);
      __syncthreads();
      for (int e = t; e < kt * r; e += kThreads) {
        const int k = e % kt, a = e / kt;
        sV[k][a] = V1[(int64_t)(k0 + k) * r + a];
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
// Scalar case (size 1, e.g. sums of squares): 256 threads take fixed strided
// slices of the partials, then a fixed-order tree in LDS.
__global__ __launch_bounds__(kThreads) void k_reduce_scalar(const double* __restrict__ partials, int nchunks,
                                                            double* __restrict__ out, double* __restrict__ out2) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int ch = threadIdx.x; ch < nchunks; ch += kThreads) s += partials[ch];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0];
    if (out2) out2[0] = red[0];
  }
}

// 16 consecutive entries x SL chunk slices per workgroup (slice sl sums chunks
// sl, sl + SL, ...); the slices are then summed in a fixed order: SL = 16
// for few chunks, 64 when there are many chunks of a small matrix (a Gram
// pass's partials), so that each thread's chain of dependent loads stays short.
template <int SL>
__global__ __launch_bounds__(16 * SL) void k_reduce(const double* __restrict__ partials, int nchunks,
                                                    int64_t size, double* __restrict__ out,
                                                    double* __restrict__ out2) {
  __shared__ double red[SL][17];
  const int el = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + el;
  double s = 0.0;
  if (e < size)
    for (int ch = sl; ch < nchunks; ch += SL) s += partials[(int64_t)ch * size + e];
  red[sl][el] = s;
  __syncthreads();
  if (sl == 0 && e < size) {
    double tot = 0.0;
    for (int k = 0; k < SL; ++k) tot += red[k][el];
    out[e] = tot;
    if (out2) out2[e] = tot;
  }
}

// First stage of a two-stage fixed-order sum for many chunks of a short vector:
// workgroup (b, s) sums chunks [s K, min((s + 1) K, nchunks)) of entries
// 16 b .. 16 b + 15 into stripes[s size + e] (the order inside a stripe as in
// k_reduce; the stripes are then summed in order by k_reduce).
__global__ __launch_bounds__(16 * 16) void k_reduce_stripe(const double* __restrict__ partials, int nchunks,
                                                           int per_stripe, int64_t size,
                                                           double* __restrict__ stripes) {
  __shared__ double red[16][17];
  const int el = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + el;
  const int c0 = blockIdx.y * per_stripe;
  const int c1 = min(nchunks, c0 + per_stripe);
  double s = 0.0;
  if (e < size)
    for (int ch = c0 + sl; ch < c1; ch += 16) s += partials[(int64_t)ch * size + e];
  red[sl][el] = s;
  __syncthreads();
  if (sl == 0 && e < size) {
    double tot = 0.0;
    for (int k = 0; k < 16; ++k) tot += red[k][el];
    stripes[(int64_t)blockIdx.y * size + e] = tot;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Row chunks of a partial-product pass: at most 1024 (chunk, column block)
// workgroups and at most 512 chunks (a narrow Gram pass over 1M x 32 FP64 ran
// 13% faster on 512 chunks than on 1024, with half the partials to reduce).
int atb_chunks(int64_t m, int n, int c) {
  (void)c;
  const int64_t tiles = (m + kAtbTR - 1) / kAtbTR;
  const int colblocks = (n + kAtbJT - 1) / kAtbJT;
  int64_t want = 1024 / colblocks;
  if (want > 512) want = 512;
  if (want < 1) want = 1;
  return (int)(tiles < want ? tiles : want);
}

template <typename TA>
static hipError_t launch_gram_narrow(const TA* A, int64_t m, int n, int layout, int64_t rpc, double* partials,
                                     int nchunks, hipStream_t st) {
  const int nb = (n + 15) / 16;
  // vector loads need 16-byte aligned column starts and run starts (rows per chunk a multiple of the run)
  constexpr int RPL = 64 / (int)sizeof(TA);
  const bool vec = layout == COL && ((uintptr_t)A % 16) == 0 && (m * (int64_t)sizeof(TA)) % 16 == 0 &&
                   rpc % RPL == 0;
#define TT_GRN(NBV, LYV, VECV)                                                                                   \
  TT_LAUNCH((k_gram_narrow<TA, NBV, LYV, VECV>), dim3(nchunks), dim3(kThreads), 0, st, A, m, n, rpc, partials)
#define TT_GRN_NB(LYV, VECV)                                                                                     \
  do {                                                                                                          \
    if (nb == 1) TT_GRN(1, LYV, VECV); else if (nb == 2) TT_GRN(2, LYV, VECV);                                  \
    else if (nb == 3) TT_GRN(3, LYV, VECV); else TT_GRN(4, LYV, VECV);                                          \
  } while (0)
  if (layout == ROW) TT_GRN_NB(ROW, false);
  else if (vec) TT_GRN_NB(COL, true);
  else TT_GRN_NB(COL, false);
#undef TT_GRN_NB
#undef TT_GRN
  return hipGetLastError();
}

hipError_t launch_atb(const void* A, int a_f32, const void* Y, int y_f32, int64_t m, int n, int c,
                      int layout, double* partials, int nchunks, hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || m < 1 || nchunks < 1) return hipErrorInvalidValue;
  const int64_t rpc = (m + nchunks - 1) / nchunks;
  // Gram passes (Y == A, c == n <= 64): both operands from the same loads; row
  // chunks rounded to whole 32-row runs (empty trailing chunks give zero partials)
  if (A == Y && a_f32 == y_f32 && c == n && n <= kAtbJT) {
    if (a_f32) return launch_gram_narrow<float>((const float*)A, m, n, layout, (rpc + 31) / 32 * 32, partials, nchunks, st);
    return launch_gram_narrow<double>((const double*)A, m, n, layout, (rpc + 31) / 32 * 32, partials, nchunks, st);
  }
  return launch_atb2(A, a_f32, Y, y_f32, m, n, c, layout, 0, partials, nchunks, st);
}

// Short A: the k range is split over the waves of a workgroup of 16 rows.
static bool ax_short(int64_t m, int n) { return (m + 63) / 64 < kAxSplitTiles && n > kAxKC; }

// Narrow A: W fits the registers of every lane (NK * ceil(c/16) <= 32 doubles, NK =
// ceil(n/4) rounded up to the instantiated 4, 8 or 16).
static int ax_nk(int n) {
  const int nk = (n + 3) / 4;
  return nk <= 4 ? 4 : (nk <= 8 ? 8 : 16);
}
static bool ax_narrow(int n, int c) { return n <= 64 && ax_nk(n) * ((c + 15) / 16) <= 32; }
constexpr int kNarrowGroups = 2048;   // workgroups of the narrow kernel (grid-stride over row blocks)

int ax_chunks(int64_t m, int n, int c) {
  if (ax_narrow(n, c)) {
    // narrow kernels: 4 waves per group, 16-row blocks (16*RB-row blocks in the vector form; the
    // same group count keeps the sum-of-squares partials independent of the form)
    const int64_t groups = ((m + 15) / 16 + 3) / 4;
    return (int)(groups < kNarrowGroups ? groups : kNarrowGroups);
  }
  if (ax_short(m, n)) return (int)((m + 15) / 16);
  const int64_t tiles = (m + 63) / 64;
  return (int)(tiles < 8192 ? tiles : 8192);
}

// The vector form of A*W needs 16-byte aligned column runs of A (and of Y for
// its RB-row stores).
template <int RB, typename TA, typename TY>
static bool ax_cv_ok(const TA* A, const TY* Y, int64_t m) {
  return ((uintptr_t)A % (RB * sizeof(TA))) == 0 && m % RB == 0 && ((uintptr_t)Y % (RB * sizeof(TY))) == 0;
}
// Row runs (RB) and W chunk width (KC) of the vector A*W, as measured fastest
// at 32768 x 512 (FP64, c = 24), 640000 x 1280 (FP64 and FP32, c = 48) and
// 2560000 x 1280 (c = 40 and 48: KC = 32 for FP64 data with c <= 48 and for
// the FP32 matrix-core form, 3-4% faster than 16): FP64 data in runs of 2
// rows, FP32 data in runs of 4 (2 where the FP64 accumulators of 4 rows would
// not fit the registers: FP64 matrix cores with c > 32).
template <typename TA, int NT, bool F32M>
struct AxvCfg {
  static constexpr int RB = sizeof(TA) == 8 ? 2 : (F32M || NT <= 2 ? 4 : 2);
  static constexpr int KC = NT <= 3 && (sizeof(TA) == 8 || RB == 2 || F32M) ? 32 : 16;
};

template <typename TA, typename TY, int LY>
static void ax_dispatch_l(const TA* A, const double* W, TY* Y, int64_t m, int n, int c, int nchunks,
                          double* sumsqA, double* sumsqY, double* rerr, hipStream_t st) {
  dim3 grid(nchunks), block(kThreads);
  if (ax_narrow(n, c)) {
    const int nk = ax_nk(n);
    constexpr int RBV = 16 / (int)sizeof(TA);
    if (LY == COL && ax_cv_ok<RBV>(A, Y, m) && ((c + 15) / 16) <= 2) {
      const int nkv = (n + 3) / 4;
#define TT_AXV(NTV, NKV) TT_LAUNCH((k_ax_narrow_v<TA, TY, NTV, NKV, RBV>), grid, block, 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr)
      if (c <= 16) { if (nkv <= 4) TT_AXV(1, 4); else if (nkv <= 8) TT_AXV(1, 8); else if (nkv <= 12) TT_AXV(1, 12); else TT_AXV(1, 16); }
      else { if (nkv <= 4) TT_AXV(2, 4); else if (nkv <= 8) TT_AXV(2, 8); else if (nkv <= 12) TT_AXV(2, 12); else TT_AXV(2, 16); }
#undef TT_AXV
      return;
    }
#define TT_AXN(NTV, NKV) TT_LAUNCH((k_ax_narrow<TA, TY, NTV, NKV, LY>), grid, block, 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr)
    if (c <= 16) { if (nk <= 4) TT_AXN(1, 4); else if (nk <= 8) TT_AXN(1, 8); else TT_AXN(1, 16); }
    else if (c <= 32) { if (nk <= 4) TT_AXN(2, 4); else if (nk <= 8) TT_AXN(2, 8); else TT_AXN(2, 16); }
    else if (c <= 48) { if (nk <= 4) TT_AXN(3, 4); else TT_AXN(3, 8); }
    else { if (nk <= 4) TT_AXN(4, 4); else TT_AXN(4, 8); }
#undef TT_AXN
    return;
  }
  if (ax_short(m, n)) {
    if (c <= 16)
      TT_LAUNCH((k_ax_kw<TA, TY, 1, LY>), grid, dim3(ax_kw_threads(1)), 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr);
    else if (c <= 32)
      TT_LAUNCH((k_ax_kw<TA, TY, 2, LY>), grid, dim3(ax_kw_threads(2)), 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr);
    else if (c <= 48)
      TT_LAUNCH((k_ax_kw<TA, TY, 3, LY>), grid, dim3(ax_kw_threads(3)), 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr);
    else
      TT_LAUNCH((k_ax_kw<TA, TY, 4, LY>), grid, dim3(ax_kw_threads(4)), 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr);
    return;
  }
  if (LY == COL && ax_cv_ok<2>(A, Y, m) && (sizeof(TA) == 8 || ax_cv_ok<4>(A, Y, m))) {
#define TT_AXC(NTV)                                                                                       \
  TT_LAUNCH((k_ax_cv<TA, TY, NTV, false, AxvCfg<TA, NTV, false>::RB, AxvCfg<TA, NTV, false>::KC>), grid, \
            block, 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr)
    if (c <= 16) TT_AXC(1); else if (c <= 32) TT_AXC(2); else if (c <= 48) TT_AXC(3); else TT_AXC(4);
#undef TT_AXC
    return;
  }
  if (c <= 16)
    TT_LAUNCH((k_ax<TA, TY, 1, LY>), grid, block, 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr);
  else if (c <= 32)
    TT_LAUNCH((k_ax<TA, TY, 2, LY>), grid, block, 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr);
  else if (c <= 48)
    TT_LAUNCH((k_ax<TA, TY, 3, LY>), grid, block, 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr);
  else
    TT_LAUNCH((k_ax<TA, TY, 4, LY>), grid, block, 0, st, A, W, Y, m, n, c, sumsqA, sumsqY, rerr);
}

template <typename TA, typename TY>
static void ax_dispatch(const TA* A, const double* W, TY* Y, int64_t m, int n, int c, int layout,
                        int nchunks, double* sumsqA, double* sumsqY, double* rerr, hipStream_t st) {
  if (layout == ROW) ax_dispatch_l<TA, TY, ROW>(A, W, Y, m, n, c, nchunks, sumsqA, sumsqY, rerr, st);
  else ax_dispatch_l<TA, TY, COL>(A, W, Y, m, n, c, nchunks, sumsqA, sumsqY, rerr, st);
}

hipError_t launch_ax(const void* A, int a_f32, const double* W, void* Y, int y_f32, int64_t m, int n,
                     int c, int layout, int nchunks, double* sumsqA, double* sumsqY, double* rerr,
                     hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || m < 1 || nchunks != ax_chunks(m, n, c)) return hipErrorInvalidValue;
  if (!a_f32 && !y_f32)
    ax_dispatch((const double*)A, W, (double*)Y, m, n, c, layout, nchunks, sumsqA, sumsqY, rerr, st);
  else if (a_f32 && !y_f32)
    ax_dispatch((const float*)A, W, (double*)Y, m, n, c, layout, nchunks, sumsqA, sumsqY, rerr, st);
  else if (a_f32 && y_f32)
    ax_dispatch((const float*)A, W, (float*)Y, m, n, c, layout, nchunks, sumsqA, sumsqY, rerr, st);
  else
    ax_dispatch((const double*)A, W, (float*)Y, m, n, c, layout, nchunks, sumsqA, sumsqY, rerr, st);
  return hipGetLastError();
}

int resid_chunks(int64_t m) {
  const int64_t tiles = (m + kResTR - 1) / kResTR;
  return (int)(tiles < 2048 ? tiles : 2048);
}

hipError_t launch_resid(const void* A, int a_f32, const void* Cr, int c_f32, const double* V1, int64_t m,
                        int n, int r, int layout, int nchunks, double* resid, hipStream_t st) {
  if (n < 1 || r < 1 || r > kCMax || m < 1 || nchunks < 1) return hipErrorInvalidValue;
  const int64_t rpc = (m + nchunks - 1) / nchunks;
  dim3 g(nchunks), b(kThreads);
  if (a_f32 && c_f32)
    TT_LAUNCH((k_resid<float, float>), g, b, 0, st, (const float*)A, (const float*)Cr, V1, m, n, r, layout, rpc, resid);
  else if (a_f32)
    TT_LAUNCH((k_resid<float, double>), g, b, 0, st, (const float*)A, (const double*)Cr, V1, m, n, r, layout, rpc, resid);
  else if (c_f32)
    TT_LAUNCH((k_resid<double, float>), g, b, 0, st, (const double*)A, (const float*)Cr, V1, m, n, r, layout, rpc, resid);
  else
    TT_LAUNCH((k_resid<double, double>), g, b, 0, st, (const double*)A, (const double*)Cr, V1, m, n, r, layout, rpc, resid);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nchunks, int64_t size, double* out,
                         double* out2, hipStream_t st, double* stripes) {
  if (size < 1 || nchunks < 1) return hipErrorInvalidValue;
  if (size == 1) {
    TT_LAUNCH(k_reduce_scalar, dim3(1), dim3(kThreads), 0, st, partials, nchunks, out, out2);
    return hipGetLastError();
  }
  const int64_t blocks = (size + 15) / 16;
  if (stripes && nchunks >= 2048 && blocks < 128) {
    // few workgroups over many chunks: two stages, kReduceStripes stripes first
    const int per = (nchunks + kReduceStripes - 1) / kReduceStripes;
    TT_LAUNCH(k_reduce_stripe, dim3((unsigned)blocks, (unsigned)kReduceStripes), dim3(16 * 16), 0, st, partials,
              nchunks, per, size, stripes);
    TT_LAUNCH(k_reduce<16>, dim3((unsigned)blocks), dim3(16 * 16), 0, st, stripes, kReduceStripes, size, out, out2);
    return hipGetLastError();
  }
  if (nchunks >= 256)
    TT_LAUNCH(k_reduce<64>, dim3((unsigned)blocks), dim3(16 * 64), 0, st, partials, nchunks, size, out, out2);
  else
    TT_LAUNCH(k_reduce<16>, dim3((unsigned)blocks), dim3(16 * 16), 0, st, partials, nchunks, size, out, out2);
  return hipGetLastError();
}

}  // namespace ttutv

namespace ttutv {

hipError_t launch_ax_lp(const void* A, int a_f32, const double* W, float* Y, int64_t m, int n, int c, int layout,
                        int bf16, hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || m < 1) return hipErrorInvalidValue;
  const int64_t tiles = (m + 63) / 64;
  dim3 grid((unsigned)(tiles < 8192 ? tiles : 8192)), block(kThreads);
#define TT_AXL(TAV, NTV, BFV)                                                                             \
  do {                                                                                                    \
    if (layout == ROW)                                                                                    \
      TT_LAUNCH((k_ax_lp<TAV, NTV, ROW, BFV>), grid, block, 0, st, (const TAV*)A, W, Y, m, n, c);         \
    else                                                                                                  \
      TT_LAUNCH((k_ax_lp<TAV, NTV, COL, BFV>), grid, block, 0, st, (const TAV*)A, W, Y, m, n, c);         \
  } while (0)
#define TT_AXL_NT(TAV, BFV)                                                                               \
  do {                                                                                                    \
    const int nt = (c + 15) / 16;                                                                         \
    if (nt == 1) TT_AXL(TAV, 1, BFV); else if (nt == 2) TT_AXL(TAV, 2, BFV);                              \
    else if (nt == 3) TT_AXL(TAV, 3, BFV); else TT_AXL(TAV, 4, BFV);                                      \
  } while (0)
#define TT_AXF(TAV, NTV)                                                                                  \
  do {                                                                                                    \
    if (layout == ROW)                                                                                    \
      TT_LAUNCH((k_ax_f32<TAV, NTV, ROW>), grid, block, 0, st, (const TAV*)A, W, Y, m, n, c);             \
    else                                                                                                  \
      TT_LAUNCH((k_ax_f32<TAV, NTV, COL>), grid, block, 0, st, (const TAV*)A, W, Y, m, n, c);             \
  } while (0)
#define TT_AXF_NT(TAV)                                                                                    \
  do {                                                                                                    \
    const int nt = (c + 15) / 16;                                                                         \
    if (nt == 1) TT_AXF(TAV, 1); else if (nt == 2) TT_AXF(TAV, 2);                                        \
    else if (nt == 3) TT_AXF(TAV, 3); else TT_AXF(TAV, 4);                                                \
  } while (0)
#define TT_AXCV(TAV)                                                                                      \
  do {                                                                                                    \
    const int64_t cvt = (m + 64 * 4 - 1) / (64 * 4);                                                      \
    dim3 g2((unsigned)(cvt < 8192 ? cvt : 8192));                                                         \
    const TAV* Ap = (const TAV*)A;                                                                        \
    const int nt = (c + 15) / 16;                                                                         \
    if (nt == 1) TT_LAUNCH((k_ax_cv<TAV, float, 1, true, 4, AxvCfg<TAV, 1, true>::KC>), g2, block, 0, st, Ap, W, Y, m, n, c, nullptr, nullptr, nullptr); \
    else if (nt == 2) TT_LAUNCH((k_ax_cv<TAV, float, 2, true, 4, AxvCfg<TAV, 2, true>::KC>), g2, block, 0, st, Ap, W, Y, m, n, c, nullptr, nullptr, nullptr); \
    else if (nt == 3) TT_LAUNCH((k_ax_cv<TAV, float, 3, true, 4, AxvCfg<TAV, 3, true>::KC>), g2, block, 0, st, Ap, W, Y, m, n, c, nullptr, nullptr, nullptr); \
    else TT_LAUNCH((k_ax_cv<TAV, float, 4, true, 4, AxvCfg<TAV, 4, true>::KC>), g2, block, 0, st, Ap, W, Y, m, n, c, nullptr, nullptr, nullptr); \
  } while (0)
  if (a_f32) {
    if (bf16) TT_AXL_NT(float, true);
    else if (layout == COL && ax_cv_ok<4>((const float*)A, Y, m)) TT_AXCV(float);
    else TT_AXF_NT(float);
  } else {
    if (bf16) TT_AXL_NT(double, true); else TT_AXF_NT(double);
  }
#undef TT_AXCV
#undef TT_AXF_NT
#undef TT_AXF
#undef TT_AXL_NT
#undef TT_AXL
  return hipGetLastError();
}

int atb_lp_chunks(int64_t m, int n) {
  return atb_chunks(m, n, 0);   // the same number of partials as the FP64 kernel (workspace bound)
}

hipError_t launch_atb_lp(const void* A, int a_f32, const float* Y, int64_t m, int n, int c, int layout,
                         double* partials, int nchunks, int bf16, hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || m < 1 || nchunks < 1) return hipErrorInvalidValue;
  int64_t rpc = (m + nchunks - 1) / nchunks;
  rpc = (rpc + 15) / 16 * 16;
  dim3 grid(nchunks, (n + kAtbJT - 1) / kAtbJT), block(kThreads);
#define TT_ATBL(TAV, NTV, BFV)                                                                               \
  do {                                                                                                       \
    if (layout == ROW)                                                                                       \
      TT_LAUNCH((k_atb_lp<TAV, NTV, ROW, BFV>), grid, block, 0, st, (const TAV*)A, Y, m, n, c, rpc, partials); \
    else                                                                                                     \
      TT_LAUNCH((k_atb_lp<TAV, NTV, COL, BFV>), grid, block, 0, st, (const TAV*)A, Y, m, n, c, rpc, partials); \
  } while (0)
#define TT_ATBL_NT(TAV, BFV)                                                                                 \
  do {                                                                                                       \
    const int nt = (c + 15) / 16;                                                                            \
    if (nt == 1) TT_ATBL(TAV, 1, BFV); else if (nt == 2) TT_ATBL(TAV, 2, BFV);                               \
    else if (nt == 3) TT_ATBL(TAV, 3, BFV); else TT_ATBL(TAV, 4, BFV);                                       \
  } while (0)
  if (a_f32) { if (bf16) TT_ATBL_NT(float, true); else TT_ATBL_NT(float, false); }
  else { if (bf16) TT_ATBL_NT(double, true); else TT_ATBL_NT(double, false); }
#undef TT_ATBL_NT
#undef TT_ATBL
  return hipGetLastError();
}

}  // namespace ttutv

namespace ttutv {

int atb2_chunks(int64_t m, int n) {
  return atb_chunks(m, n, 0);   // no more partials than the 64-column kernel (workspace bound)
}

bool fused_ata_ok(int a_f32, int64_t m, int n, int c, int layout) {
  return !a_f32 && layout == COL && m >= 1 && n >= 1 && n <= kFaMaxN && c >= 1 && c <= 32 &&
         (int64_t)n * c <= kFaMaxNC;
}

// one block per compute unit, at most one per row tile
int fused_ata_blocks(int64_t m) {
  const int64_t tiles = (m + kFaTR - 1) / kFaTR;
  return (int)(tiles < 256 ? tiles : 256);
}

hipError_t launch_fused_ata(const double* A, const double* X, int64_t m, int n, int c, double* partials, int nblocks,
                            hipStream_t st) {
  if (!fused_ata_ok(0, m, n, c, COL) || nblocks != fused_ata_blocks(m)) return hipErrorInvalidValue;
  if (c <= 16)
    TT_LAUNCH((k_fused_ata<1>), dim3(nblocks), dim3(kFaThreads), 0, st, A, X, m, n, c, partials);
  else
    TT_LAUNCH((k_fused_ata<2>), dim3(nblocks), dim3(kFaThreads), 0, st, A, X, m, n, c, partials);
  return hipGetLastError();
}

hipError_t launch_atb2(const void* A, int a_f32, const void* Y, int y_f32, int64_t m, int n, int c, int layout,
                       int f32_mma, double* partials, int nchunks, hipStream_t st) {
  if (n < 1 || c < 1 || c > kCMax || m < 1 || nchunks < 1) return hipErrorInvalidValue;
  int64_t rpc = (m + nchunks - 1) / nchunks;
  // vector loads: column-major A with 16-byte aligned columns, chunks of whole
  // 32-row tiles (the row chunks are rounded up; trailing chunks may be empty
  // and then write zero partials)
  const int64_t vl = a_f32 ? 4 : 2;
  const bool vec = layout == COL && ((uintptr_t)A % 16) == 0 && m % vl == 0;
  if (vec) rpc = (rpc + kAtb2TR - 1) / kAtb2TR * kAtb2TR;
  // one workgroup per (chunk, column block) pair, rounded up to whole XCD shares
  const int64_t npairs = (int64_t)nchunks * ((n + kAtb2JB - 1) / kAtb2JB);
  if (npairs > 0x7ffffff8LL) return hipErrorInvalidValue;
  dim3 grid((unsigned)((npairs + 7) / 8 * 8)), block(kAtb2Threads);
#define TT_A2(TAV, TYV, NTV, F32V)                                                                           \
  do {                                                                                                       \
    if (layout == ROW)                                                                                       \
      TT_LAUNCH((k_atb2<TAV, TYV, NTV, ROW, F32V, false>), grid, block, 0, st, (const TAV*)A, (const TYV*)Y, m, \
                n, c, rpc, nchunks, partials);                                                               \
    else if (vec)                                                                                            \
      TT_LAUNCH((k_atb2<TAV, TYV, NTV, COL, F32V, true>), grid, block, 0, st, (const TAV*)A, (const TYV*)Y, m, \
                n, c, rpc, nchunks, partials);                                                               \
    else                                                                                                     \
      TT_LAUNCH((k_atb2<TAV, TYV, NTV, COL, F32V, false>), grid, block, 0, st, (const TAV*)A, (const TYV*)Y, m, \
                n, c, rpc, nchunks, partials);                                                               \
  } while (0)
#define TT_A2_NT(TAV, TYV, F32V)                                                                              \
  do {                                                                                                       \
    const int nt = (c + 15) / 16;                                                                            \
    if (nt == 1) TT_A2(TAV, TYV, 1, F32V); else if (nt == 2) TT_A2(TAV, TYV, 2, F32V);                       \
    else if (nt == 3) TT_A2(TAV, TYV, 3, F32V); else TT_A2(TAV, TYV, 4, F32V);                               \
  } while (0)
  if (f32_mma) {
    if (!a_f32 || !y_f32) return hipErrorInvalidValue;   // FP32 products only on FP32 data
    TT_A2_NT(float, float, true);
  } else if (!a_f32 && !y_f32) TT_A2_NT(double, double, false);
  else if (a_f32 && y_f32) TT_A2_NT(float, float, false);
  else if (a_f32) TT_A2_NT(float, double, false);
  else TT_A2_NT(double, float, false);
#undef TT_A2_NT
#undef TT_A2
  return hipGetLastError();
}

}  // namespace ttutv
