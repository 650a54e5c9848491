// The carry of a Gram-mode step and the first sketch product of the next
// (sketched) step in one pass over the Gram-mode step's unfolding, for the
// right-to-left sweep (column-major unfoldings, Alg. 3).
//
// Step k's unfolding A1 (m1 x n1, n1 <= 64) gives the carry C = A1 V1
// (m1 x r).  The next unfolding is A2 = reshape(C, [m2, I r]) with m1 = m2 I:
// column i + I b of A2 is rows [i m2, (i+1) m2) of column b of C, and its
// first sketch product is Y = A2 G (G: I r x c).  Splitting A1 into its I row
// slabs A1_i (m2 x n1),
//     Y = sum_b sum_i C_i(:, b) G(i + I b, :) = sum_i A1_i H_i,
//     H_i = V1 G_i (n1 x c),  G_i(b, :) = G(i + I b, :),
// so both products take the same A1 operand: the pass that writes the carry
// also forms Y, and the next step starts from it instead of reading the carry
// (the largest unfolding of the sweep after the first) once more.  H (I x n1
// x c) is formed first by k_sketch_fold.
#include "tt_internal.h"

namespace ttutv {
namespace {

constexpr int kCsThreads = 256;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double cs_block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

// H[(i n1 + k) c + j] = sum_{b < r} V1[k r + b] G[(i + I b) c + j]   (V1 and G k-major)
__global__ __launch_bounds__(kCsThreads) void k_sketch_fold(const double* __restrict__ V1,
                                                            const double* __restrict__ G, double* __restrict__ H,
                                                            int I, int n1, int r, int c) {
  const int64_t total = (int64_t)I * n1 * c;
  for (int64_t e = (int64_t)blockIdx.x * kCsThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kCsThreads) {
    const int j = (int)(e % c);
    const int64_t ik = e / c;
    const int k = (int)(ik % n1), i = (int)(ik / n1);
    double s = 0.0;
    for (int b = 0; b < r; ++b) s = fma(V1[(int64_t)k * r + b], G[((int64_t)i + (int64_t)I * b) * c + j], s);
    H[e] = s;
  }
}

// One workgroup = 4 waves = a tile of 64 RB rows of every slab (rows
// tile*TR .. tile*TR + TR - 1 of A1_i for i = 0 .. I-1).  Lane li of wave w
// owns the RB consecutive rows 16 RB w + RB li + (0 .. RB-1) of the tile and
// loads them with one vector load per column; MFMA row block rb holds rows
// RB li + rb.  V1 (n1 x r) sits in LDS for the launch; H_i is staged per slab,
// double-buffered, the next slab's A1 rows are loaded into the other register
// buffer while the current slab runs on the matrix cores (every load is
// issued unconditionally, at clamped addresses: rows past m2 fall in the tile
// rows never stored, columns past n1 meet zero rows of V1 and H).  The carry
// rows of a slab are written as they are formed (one vector store per lane
// and column); Y's rows are accumulated over the slabs in registers and
// written at the end.  The carry's sum of squares (and, for an FP32 carry,
// the sum of squares of its rounding error) is left as per-workgroup partials.
// NS: k-steps (4 (NS - 1) < n1 <= 4 NS), NT1 and NT2: column tiles of the carry
// and of Y, all fixed at compile time so that the matrix-core blocks carry no
// branches; FS: the sketch product on FP32 matrix cores (operands rounded to
// FP32, FP32 accumulation), else FP64.
template <typename TA, typename TC, typename TY, int NS, int NT1, int NT2, int RB, bool FS>
__global__ __launch_bounds__(kCsThreads, 1) void k_carry_sketch(const TA* __restrict__ A, int64_t m2, int I,
                                                                int n1, const double* __restrict__ V1, int r,
                                                                const double* __restrict__ H, int c,
                                                                TC* __restrict__ C, TY* __restrict__ Y,
                                                                double* __restrict__ sumsqC,
                                                                double* __restrict__ rerr) {
  constexpr int TR = 4 * 16 * RB;
  constexpr int LV = NT1 * 16 + 1;           // padded LDS rows
  constexpr int LH = NT2 * 16 + 1;
  typedef typename std::conditional<FS, float, double>::type TS;   // sketch operand type
  typedef typename std::conditional<FS, f4, d4>::type acc2_t;
  typedef TA vec_t __attribute__((ext_vector_type(RB)));
  typedef TC cvec_t __attribute__((ext_vector_type(RB)));
  typedef TY yvec_t __attribute__((ext_vector_type(RB)));
  __shared__ double sV[4 * NS][LV];
  __shared__ TS sH[2][4 * NS][LH];
  __shared__ double sh[8];
  constexpr int NHS = (4 * NS * NT2 * 16 + kCsThreads - 1) / kCsThreads;   // H entries staged per thread
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t m1 = m2 * I;
  for (int e = t; e < 4 * NS * NT1 * 16; e += kCsThreads) {
    const int k = e / (NT1 * 16), col = e % (NT1 * 16);
    sV[k][col] = (k < n1 && col < r) ? V1[(int64_t)k * r + col] : 0.0;
  }
  double ssc = 0.0, sse = 0.0;
  const int64_t ntiles = (m2 + TR - 1) / TR;
  auto load_h = [&](int i, TS* dst) {
    const double* Hi = H + (int64_t)i * n1 * c;
#pragma unroll
    for (int u = 0; u < NHS; ++u) {
      const int e = t + kCsThreads * u;
      const int k = e / (NT2 * 16), col = e % (NT2 * 16);
      const bool ok = e < 4 * NS * NT2 * 16 && k < n1 && col < c;
      const double v = Hi[ok ? (int64_t)k * c + col : 0];
      dst[u] = ok ? (TS)v : (TS)0;
    }
  };
  auto store_h = [&](const TS* src, int buf) {
#pragma unroll
    for (int u = 0; u < NHS; ++u) {
      const int e = t + kCsThreads * u;
      if (e < 4 * NS * NT2 * 16) sH[buf][e / (NT2 * 16)][e % (NT2 * 16)] = src[u];
    }
  };
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * TR + 16 * RB * w + RB * li;   // slab-relative first row of this lane
    const int64_t rowc = row < m2 - RB ? row : m2 - RB;      // m2 is a multiple of RB
    auto load_a = [&](int i, vec_t* a) {
      const TA* p = A + (int64_t)i * m2 + rowc;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int k = 4 * s + g;
        const int kc = k < n1 ? k : n1 - 1;
        a[s] = *reinterpret_cast<const vec_t*>(p + (int64_t)kc * m1);
      }
    };
    acc2_t acc2[RB][NT2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int u = 0; u < NT2; ++u) acc2[rb][u] = acc2_t{0, 0, 0, 0};
    // slab i: the carry rows (written now) and the slab's share of Y
    auto slab = [&](const vec_t* a, int buf, int i) {
      d4 acc1[RB][NT1];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int q = 0; q < NT1; ++q) acc1[rb][q] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        double bv[NT1];
        TS bh[NT2];
#pragma unroll
        for (int q = 0; q < NT1; ++q) bv[q] = sV[4 * s + g][16 * q + li];
#pragma unroll
        for (int u = 0; u < NT2; ++u) bh[u] = sH[buf][4 * s + g][16 * u + li];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const double x = (double)a[s][rb];
#pragma unroll
          for (int q = 0; q < NT1; ++q) acc1[rb][q] = mfma64(x, bv[q], acc1[rb][q]);
#pragma unroll
          for (int u = 0; u < NT2; ++u) {
            if constexpr (FS) acc2[rb][u] = mfma32((float)a[s][rb], bh[u], acc2[rb][u]);
            else acc2[rb][u] = mfma64(x, bh[u], acc2[rb][u]);
          }
        }
      }
      // carry: register v of a lane holds MFMA row g + 4v, i.e. tile rows RB (g + 4v) + rb
#pragma unroll
      for (int q = 0; q < NT1; ++q) {
        const int col = 16 * q + li;
        if (col >= r) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r0 = tile * TR + 16 * RB * w + RB * (g + 4 * v);
          cvec_t cv;
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const double sv = acc1[rb][q][v];
            const TC y = (TC)sv;
            cv[rb] = y;
            if (r0 + rb < m2) {
              const double yd = (double)y;
              ssc = fma(yd, yd, ssc);
              const double er = sv - yd;
              sse = fma(er, er, sse);
            }
          }
          TC* dst = C + (int64_t)i * m2 + r0 + (int64_t)col * m1;
          if (r0 + RB <= m2) {
            *reinterpret_cast<cvec_t*>(dst) = cv;
          } else {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
              if (r0 + rb < m2) dst[rb] = cv[rb];
          }
        }
      }
    };
    vec_t a0[NS], a1[NS];
    TS hn[NHS];
    __syncthreads();   // sV written; the previous tile's reads of sH are done
    load_h(0, hn);
    store_h(hn, 0);
    load_a(0, a0);
    __syncthreads();
    for (int i = 0; i < I; i += 2) {
      // slab i in a0 / sH[0]; slab i + 1 in a1 / sH[1] (past the last slab: an unused reload)
      const bool more1 = i + 1 < I;
      load_h(more1 ? i + 1 : i, hn);
      load_a(more1 ? i + 1 : i, a1);
      slab(a0, 0, i);
      store_h(hn, 1);
      __syncthreads();
      if (!more1) break;
      const bool more2 = i + 2 < I;
      load_h(more2 ? i + 2 : i + 1, hn);
      load_a(more2 ? i + 2 : i + 1, a0);
      slab(a1, 1, i + 1);
      store_h(hn, 0);
      __syncthreads();
    }
    // Y rows of the tile: register v holds MFMA row g + 4v (FP64) or 4g + v (FP32)
#pragma unroll
    for (int u = 0; u < NT2; ++u) {
      const int col = 16 * u + li;
      if (col >= c) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rho = FS ? 4 * g + v : g + 4 * v;
        const int64_t r0 = tile * TR + 16 * RB * w + RB * rho;
        yvec_t yv;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) yv[rb] = (TY)acc2[rb][u][v];
        TY* dst = Y + r0 + (int64_t)col * m2;
        if (r0 + RB <= m2) {
          *reinterpret_cast<yvec_t*>(dst) = yv;
        } else {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            if (r0 + rb < m2) dst[rb] = yv[rb];
        }
      }
    }
  }
  {
    const double s = cs_block_sum(ssc, sh);
    if (t == 0) sumsqC[blockIdx.x] = s;
  }
  if (rerr) {
    const double s = cs_block_sum(sse, sh);
    if (t == 0) rerr[blockIdx.x] = s;
  }
}

constexpr int kCsMaxGroups = 2048;

template <typename TA, typename TC, typename TY, int NS, int NT1, int NT2, bool FS>
hipError_t cs_go(const TA* A, int64_t m2, int I, int n1, const double* V1, int r, const double* H, int c, TC* C, TY* Y,
                 double* sumsqC, double* rerr, int groups, hipStream_t st) {
  // rows per lane: runs of 4 for FP32 data with FP32 sketch accumulators, else 2 (the FP64
  // accumulators of 4 rows do not fit the registers)
  constexpr int RB = (sizeof(TA) == 4 && FS) ? 4 : 2;
  TT_LAUNCH((k_carry_sketch<TA, TC, TY, NS, NT1, NT2, RB, FS>), dim3(groups), dim3(kCsThreads), 0, st, A, m2, I, n1,
            V1, r, H, c, C, Y, sumsqC, rerr);
  return hipGetLastError();
}

template <typename TA, typename TC, typename TY, int NS, bool FS>
hipError_t cs_tiles(const TA* A, int64_t m2, int I, int n1, const double* V1, int r, const double* H, int c, TC* C,
                    TY* Y, double* sumsqC, double* rerr, int groups, hipStream_t st) {
  const bool two = r > 16;
  if (c <= 32) {
    if (two) return cs_go<TA, TC, TY, NS, 2, 2, FS>(A, m2, I, n1, V1, r, H, c, C, Y, sumsqC, rerr, groups, st);
    return cs_go<TA, TC, TY, NS, 1, 2, FS>(A, m2, I, n1, V1, r, H, c, C, Y, sumsqC, rerr, groups, st);
  }
  if (two) return cs_go<TA, TC, TY, NS, 2, 3, FS>(A, m2, I, n1, V1, r, H, c, C, Y, sumsqC, rerr, groups, st);
  return cs_go<TA, TC, TY, NS, 1, 3, FS>(A, m2, I, n1, V1, r, H, c, C, Y, sumsqC, rerr, groups, st);
}

// k-steps: n1 <= 32, 40, 48, or 64 (the last with FP32 sketch operands only: LDS)
template <typename TA, typename TC, typename TY, bool FS>
hipError_t cs_launch(const TA* A, int64_t m2, int I, int n1, const double* V1, int r, const double* H, int c,
                     TC* C, TY* Y, double* sumsqC, double* rerr, int groups, hipStream_t st) {
  if (n1 <= 32) return cs_tiles<TA, TC, TY, 8, FS>(A, m2, I, n1, V1, r, H, c, C, Y, sumsqC, rerr, groups, st);
  if (n1 <= 40) return cs_tiles<TA, TC, TY, 10, FS>(A, m2, I, n1, V1, r, H, c, C, Y, sumsqC, rerr, groups, st);
  if (n1 <= 48) return cs_tiles<TA, TC, TY, 12, FS>(A, m2, I, n1, V1, r, H, c, C, Y, sumsqC, rerr, groups, st);
  if constexpr (FS) return cs_tiles<TA, TC, TY, 16, FS>(A, m2, I, n1, V1, r, H, c, C, Y, sumsqC, rerr, groups, st);
  return hipErrorInvalidValue;
}

}  // namespace

static int cs_rows_per_lane(int a_f32, int c_f32) { return (a_f32 && c_f32) ? 4 : 2; }

int carry_sketch_groups(int64_t m2, int a_f32, int c_f32) {
  const int RB = cs_rows_per_lane(a_f32, c_f32);
  const int64_t tiles = (m2 + 64 * RB - 1) / (64 * RB);
  return (int)(tiles < kCsMaxGroups ? tiles : kCsMaxGroups);
}

bool carry_sketch_ok(const void* A, int a_f32, const void* C, int c_f32, const void* Y, int64_t m2, int I, int n1,
                     int r, int c) {
  const int RB = cs_rows_per_lane(a_f32, c_f32);
  const size_t sa = a_f32 ? 4 : 8, sc = c_f32 ? 4 : 8;
  return n1 >= 1 && n1 <= (c_f32 ? 64 : 48) && r >= 1 && r <= 32 && c >= 1 && c <= 48 && I >= 1 && m2 >= RB &&
         m2 % RB == 0 && (a_f32 || !c_f32) &&
         (uintptr_t)A % (RB * sa) == 0 && (uintptr_t)C % (RB * sc) == 0 && (uintptr_t)Y % (RB * sc) == 0;
}

hipError_t launch_sketch_fold(const double* V1, const double* G, double* H, int I, int n1, int r, int c,
                              hipStream_t st) {
  const int64_t total = (int64_t)I * n1 * c;
  const int64_t b = (total + kCsThreads - 1) / kCsThreads;
  TT_LAUNCH(k_sketch_fold, dim3((unsigned)(b < 1024 ? b : 1024)), dim3(kCsThreads), 0, st, V1, G, H, I, n1, r, c);
  return hipGetLastError();
}

// FP64 form: FP64 carry and FP64 Y; mixed form (c_f32, FP32 input): FP32 carry,
// FP32 Y from the FP32 matrix cores.
hipError_t launch_carry_sketch(const void* A, int a_f32, int64_t m2, int I, int n1, const double* V1, int r,
                               const double* H, int c, void* C, int c_f32, void* Y, double* sumsqC, double* rerr,
                               int groups, hipStream_t st) {
  if (!carry_sketch_ok(A, a_f32, C, c_f32, Y, m2, I, n1, r, c) || groups < 1) return hipErrorInvalidValue;
  if (a_f32 && c_f32)
    return cs_launch<float, float, float, true>((const float*)A, m2, I, n1, V1, r, H, c, (float*)C, (float*)Y,
                                                sumsqC, rerr, groups, st);
  if (a_f32)
    return cs_launch<float, double, double, false>((const float*)A, m2, I, n1, V1, r, H, c, (double*)C, (double*)Y,
                                                   sumsqC, rerr, groups, st);
  return cs_launch<double, double, double, false>((const double*)A, m2, I, n1, V1, r, H, c, (double*)C, (double*)Y,
                                                  sumsqC, rerr, groups, st);
}

}  // namespace ttutv
