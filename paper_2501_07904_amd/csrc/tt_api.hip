// Host side of libttutv: argument checks, the per-step plan of the sweep,
// the kernel sequence of every truncated UTV step, and the C ABI.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/ttutv.h"
#include "tt_internal.h"

using namespace ttutv;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_OK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(TT_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

// ---- optional per-launch timing with HIP events on the caller's stream ----
enum KClass { KC_ATB = 0, KC_AX = 1, KC_GRAM_Y = 2, KC_CARRY = 3, KC_RESID = 4, KC_REDUCE = 5, KC_SMALL = 6,
              KC_ATA = 7, KC_DEFL = 8 };
const char* const kClassNames[TT_NKCLASS] = {"tall_atb", "tall_ax", "gram_y", "carry", "resid", "reduce", "small",
                                             "tall_ata", "defl_pass"};

thread_local std::vector<hipEvent_t> g_events;
}  // namespace

namespace ttutv {
thread_local LaunchTiming g_launch_timing;
}

namespace {

struct Prof {
  bool on = false;
  int mask = 0;     // classes whose launches are timed
  hipStream_t st = nullptr;
  size_t next = 0;
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<Rec> recs;
  hipError_t event(hipEvent_t* e) {
    if (next == g_events.size()) {
      hipEvent_t x;
      hipError_t rc = hipEventCreate(&x);
      if (rc != hipSuccess) return rc;
      g_events.push_back(x);
    }
    *e = g_events[next++];
    return hipSuccess;
  }
};

#define LAUNCH(P, cls, nbytes, nflops, expr)                                        \
  do {                                                                             \
    hipEvent_t ea_ = nullptr, eb_ = nullptr;                                       \
    const bool tm_ = (P).on && (((P).mask >> (cls)) & 1);                          \
    if (tm_) {                                                                     \
      HIP_OK((P).event(&ea_));                                                     \
      HIP_OK((P).event(&eb_));                                                     \
      g_launch_timing = LaunchTiming{ea_, eb_};                                    \
    }                                                                              \
    const hipError_t le_ = (expr);                                                 \
    g_launch_timing = LaunchTiming{};                                              \
    HIP_OK(le_);                                                                   \
    if (tm_) (P).recs.push_back({(cls), ea_, eb_, (double)(nbytes), (double)(nflops)}); \
  } while (0)

// One truncated UTV step of the sweep, in the tall frame: the m x n matrix A
// whose n columns are the core side.
struct Step {
  int core;        // 1-based index of the core this step produces
  int unfolding;   // 1-based index k of the unfolding A_k it factorises
  int64_t m;       // long side
  int n;           // core side: r_{k-1} I_k (L2R) or I_k r_k (R2L)
  int layout;      // ROW (L2R) or COL (R2L)
  int n_mode, n_rank, mode_fastest;
  int r;           // fixed rank (clamped) or the cap in eps mode
  int ell;
  bool gram;       // n <= kGramMax: A^T A formed in one pass
};

struct Problem {
  int d;
  int64_t dims[TT_MAX_D];
  bool fixed;
  int64_t ranks[TT_MAX_D + 1];  // fixed: given ranks; eps: caps
  double eps;
  double eps_rule;   // eps the per-step rank rule targets (eps less the FP32 carry budget, mixed forms)
  tt_sweep sweep;
  tt_variant variant;
  tt_dtype dtype;
  tt_opts o;
  double w[TT_MAX_D];
  bool alg4;
  bool mixed;   // carries and power iterates stored in FP32
  int bf16;     // mixed form with BF16 power products
  bool defl;    // deflation inner kernel (one core-side vector at a time)
};

int64_t prod(const int64_t* v, int a, int b) {  // v[a] * ... * v[b-1]
  int64_t p = 1;
  for (int i = a; i < b; ++i) p *= v[i];
  return p;
}

int check_args(int d, const int64_t* dims, const int64_t* ranks, double eps, tt_sweep sweep,
               tt_variant variant, tt_dtype dtype, const tt_opts* opts, Problem& P) {
  if (d < 2 || d > TT_MAX_D) return fail(TT_EINVAL, "d = %d outside [2, %d]", d, TT_MAX_D);
  if (!dims) return fail(TT_EINVAL, "dims is NULL");
  if (sweep != TT_L2R && sweep != TT_R2L) return fail(TT_EINVAL, "bad sweep %d", (int)sweep);
  if (variant != TT_ULV && variant != TT_URV && variant != TT_SVD)
    return fail(TT_EINVAL, "bad variant %d", (int)variant);
  if (dtype != TT_F64 && dtype != TT_F32) return fail(TT_EINVAL, "bad dtype %d", (int)dtype);
  P.d = d;
  for (int k = 0; k < d; ++k) {
    if (dims[k] < 1 || dims[k] >= (1 << 16))
      return fail(TT_EINVAL, "dims[%d] = %lld outside [1, 65535]", k, (long long)dims[k]);
    P.dims[k] = dims[k];
  }
  if (opts) P.o = *opts; else tt_default_opts(&P.o);
  if (P.o.q < 0 || P.o.q > 64) return fail(TT_EINVAL, "q = %d outside [0, 64]", P.o.q);
  if (P.o.oversample < 0 || P.o.oversample > TT_MAX_ELL)
    return fail(TT_EINVAL, "oversample = %d outside [0, %d]", P.o.oversample, TT_MAX_ELL);
  if (P.o.max_rank < 0) return fail(TT_EINVAL, "max_rank < 0");
  if (P.o.prec != TT_PREC_FP64 && P.o.prec != TT_PREC_MIXED && P.o.prec != TT_PREC_MIXED_BF16)
    return fail(TT_EINVAL, "bad prec %d", P.o.prec);
  if (P.o.fuse_ata != 0 && P.o.fuse_ata != 1) return fail(TT_EINVAL, "fuse_ata = %d is not 0 or 1", P.o.fuse_ata);
  if (P.o.orth != TT_ORTH_HOUSEHOLDER && P.o.orth != TT_ORTH_CHOLQR)
    return fail(TT_EINVAL, "orth = %d is not a tt_orth value", P.o.orth);
  if (P.o.inner != TT_INNER_SKETCH && P.o.inner != TT_INNER_DEFLATION)
    return fail(TT_EINVAL, "inner = %d is not a tt_inner value", P.o.inner);
  P.mixed = (P.o.prec != TT_PREC_FP64);
  P.bf16 = (P.o.prec == TT_PREC_MIXED_BF16) ? 1 : 0;
  P.sweep = sweep;
  P.variant = variant;
  P.dtype = dtype;
  P.alg4 = (sweep == TT_R2L && variant == TT_ULV);
  P.defl = (P.o.inner == TT_INNER_DEFLATION);
  if (P.defl) {
    if (P.alg4 || variant == TT_SVD)
      return fail(TT_EINVAL, "the deflation inner kernel keeps the core side orthonormal: not with %s",
                  P.alg4 ? "Alg. 4 (ULV right to left)" : "TT_SVD");
    if (P.mixed) return fail(TT_EINVAL, "the deflation inner kernel runs in the FP64 form only");
    if (P.o.q < 1) return fail(TT_EINVAL, "the deflation inner kernel needs q >= 1 power steps per vector");
  }
  P.fixed = ranks != nullptr;
  if (P.fixed) {
    if (ranks[0] != 1 || ranks[d] != 1) return fail(TT_EINVAL, "ranks must have r_0 = r_d = 1");
    for (int k = 0; k <= d; ++k) {
      if (ranks[k] < 1) return fail(TT_EINVAL, "ranks[%d] = %lld < 1", k, (long long)ranks[k]);
      P.ranks[k] = ranks[k];
    }
    P.eps = 0.0;
  } else {
    if (!(eps >= 0.0) || !isfinite(eps)) return fail(TT_EINVAL, "eps must be finite and >= 0");
    P.eps = eps;
    const int cap = P.o.max_rank > 0 ? std::min(P.o.max_rank, TT_MAX_ELL) : TT_MAX_ELL;
    for (int k = 0; k <= d; ++k) P.ranks[k] = (k == 0 || k == d) ? 1 : cap;
    double sw = 0.0;
    for (int k = 0; k < d - 1; ++k) {
      double wk;
      if (P.o.weights) {
        wk = P.o.weights[k];
        if (!(wk >= 0.0) || !isfinite(wk)) return fail(TT_EINVAL, "weights[%d] invalid", k);
      } else {
        wk = P.alg4 ? 1.0 / (d - 1) : 1.0 / sqrt((double)(d - 1));
      }
      P.w[k] = wk;
      sw += wk * wk;
    }
    if (P.o.weights && fabs(sw - 1.0) > 1e-9) return fail(TT_EINVAL, "sum of squared weights is %g, not 1", sw);
    // Mixed forms store the d-2 intermediate carries in FP32.  Rounding to
    // nearest perturbs carry k by rho_k <= 2^-24 ||carry_k|| <= 2^-24 ||A|| (the
    // carries are orthogonal projections of the unfoldings, hence no larger than
    // A, up to the earlier rho), and the reported bound is sqrt(sum delta^2) +
    // sum rho (sum delta + sum rho for Alg. 4).  The steps' rank rule therefore
    // aims at eps less this a-priori budget, so that the bound stays <= eps.
    P.eps_rule = P.eps;
    if (P.mixed) {
      const double budget = (double)(d - 2) * ldexp(1.0, -24) * 1.001;
      P.eps_rule = P.eps - budget;
      if (d > 2 && !(P.eps_rule > 0.0))
        return fail(TT_EINVAL, "eps = %g is not above the FP32 carry rounding budget %g of the mixed form", P.eps,
                    budget);
    }
  }
  return TT_OK;
}

// Shapes of every step.  For eps mode the ranks are the caps, so the shapes
// are upper bounds used to size buffers; run-time shapes are re-derived.
int plan_steps(const Problem& P, const int64_t* rk /* r_0..r_d to assume */, std::vector<Step>& S,
               int64_t* used_ranks) {
  const int d = P.d;
  S.clear();
  int64_t r[TT_MAX_D + 1];
  for (int k = 0; k <= d; ++k) r[k] = rk[k];
  if (P.sweep == TT_L2R) {
    r[0] = 1;
    for (int k = 1; k <= d - 1; ++k) {
      Step s{};
      s.core = k;
      s.unfolding = k;
      const int64_t n = r[k - 1] * P.dims[k - 1];
      const int64_t m = prod(P.dims, k, d);
      s.m = m;
      s.n = (int)n;
      s.layout = ROW;
      s.n_mode = (int)P.dims[k - 1];
      s.n_rank = (int)r[k - 1];
      s.mode_fastest = 0;
      int64_t rr = std::min<int64_t>(r[k], std::min<int64_t>(n, m));
      s.r = (int)rr;
      r[k] = rr;
      S.push_back(s);
    }
  } else {
    r[d] = 1;
    for (int k = d; k >= 2; --k) {
      Step s{};
      s.core = k;
      s.unfolding = k - 1;
      const int64_t n = P.dims[k - 1] * r[k];
      const int64_t m = prod(P.dims, 0, k - 1);
      s.m = m;
      s.n = (int)n;
      s.layout = COL;
      s.n_mode = (int)P.dims[k - 1];
      s.n_rank = (int)r[k];
      s.mode_fastest = 1;
      int64_t rr = std::min<int64_t>(r[k - 1], std::min<int64_t>(n, m));
      s.r = (int)rr;
      r[k - 1] = rr;
      S.push_back(s);
    }
  }
  if (used_ranks)
    for (int k = 0; k <= d; ++k) used_ranks[k] = r[k];
  return TT_OK;
}

int step_ell(const Problem& P, const Step& s, int ell_hint) {
  const int64_t lim = std::min<int64_t>(s.n, s.m);
  int64_t ell;
  // the deflation search: the fixed rank, or at most TT_MAX_ELL vectors (s.r is
  // the cap in eps mode)
  if (P.defl) return (int)std::min<int64_t>(std::min<int64_t>(s.r, lim), TT_MAX_ELL);
  // TT-SVD: the exact step (ell = n, G = I) up to n = 64; wider core sides take
  // subspace iteration on the leading 64 directions (kSvdPowerSteps power steps)
  if (P.variant == TT_SVD) ell = std::min<int64_t>(lim, TT_MAX_ELL);
  else if (P.fixed) ell = std::min<int64_t>((int64_t)s.r + P.o.oversample, lim);
  else ell = std::min<int64_t>(ell_hint, lim);
  return (int)ell;
}

bool step_gram(const Problem& P, const Step& s) { return !P.alg4 && s.n <= kGramMax; }

// Power steps of a TT-SVD step whose core side exceeds 64: subspace iteration
// with ell = 64 columns converges to the leading singular subspace by a factor
// (s_65 / s_r)^2 per step, so 30 steps fix it to rounding when s_65 <= 0.54 s_r.
constexpr int kSvdPowerSteps = 30;

int power_steps(const Problem& P) { return P.variant == TT_SVD ? kSvdPowerSteps : P.o.q; }

// ---- workspace layout ------------------------------------------------------
struct Work {
  double* carry[2];
  double* Y;
  double* U;   // second long-side buffer (Alg. 4 orthonormalisation)
  double* X;
  double* M;
  double* part;
  int64_t part_len;   // doubles in part
  double* H;
  double* K;
  double* V1;
  double* W;
  double* normA2;
  double* cpart;   // a carry's per-workgroup sums of squares, summed by the next step's solve
  double* fold;    // H_i = V1 G_i of a carry pass that also forms the next sketch
  int64_t fold_len;
  StepRec* recs;
  DeflState* dstate;
  size_t bytes;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kCarryParts = 8192;   // bound on the per-workgroup partials of one A*W pass

struct Sizes {
  int64_t carry, Y, U, X, part, V1, fold;
};

// Upper bounds over every step (and every ell a prescribed-accuracy step may grow to).
Sizes size_bounds(const Problem& P, const std::vector<Step>& S) {
  Sizes z{1, 1, 1, 1, 1, 1, 1};
  for (size_t i = 0; i < S.size(); ++i) {
    const Step& s = S[i];
    const int64_t lim = std::min<int64_t>(std::min<int64_t>(s.n, s.m), TT_MAX_ELL);
    const int ellmax = P.fixed ? step_ell(P, s, 0) : (int)lim;
    if (i + 1 < S.size()) z.carry = std::max(z.carry, s.m * (int64_t)s.r);
    // H_i = V1 G_i for a carry pass that forms the next step's first sketch (right-to-left,
    // a step with n <= 64 before a sketched one; sketch width <= 48)
    if (i + 1 < S.size() && P.sweep == TT_R2L && !P.alg4 && !P.o.separate_sketch)
      z.fold = std::max(z.fold, (int64_t)S[i + 1].n_mode * std::min<int64_t>(s.n, kGramMax) * 48);
    z.V1 = std::max(z.V1, (int64_t)s.n * s.r);
    const int c = std::max(1, std::min(ellmax, (int)kCMax));
    if (P.defl && !step_gram(P, s)) {
      // the deflation search: V (n x cap) and the iterate in X, the reduced pass
      // [z, ||A x||^2, ||A w||^2, ||A||^2] in M, per-workgroup pass partials in part
      z.X = std::max(z.X, (int64_t)s.n * (c + 1) + 3);
      // (+ the first-stage stripes of their two-stage reduction), for any n up to
      // the planned one
      z.part = std::max(z.part, defl_pass_scratch(s.m, s.n, s.layout));
    } else if (step_gram(P, s)) {
      z.part = std::max(z.part, (int64_t)atb_chunks(s.m, s.n, s.n) * s.n * s.n);
    } else {
      z.Y = std::max(z.Y, s.m * (int64_t)c);
      z.X = std::max(z.X, (int64_t)s.n * c);
      for (int cc = 1; cc <= c; ++cc) {   // reused by the orthonormalisation of a tall n x cc iterate
        z.part = std::max(z.part, orth_scratch(s.n, cc));
        if (P.o.orth == TT_ORTH_CHOLQR && cc <= s.n) z.part = std::max(z.part, orth_cholqr_scratch(s.n, cc));
      }
      z.part = std::max(z.part, (int64_t)atb_chunks(s.m, s.n, c) * s.n * c);
      if (P.o.fuse_ata && s.layout == COL && s.n <= 512)   // one-pass power products
        z.part = std::max(z.part, (int64_t)fused_ata_blocks(s.m) * s.n * std::min(c, 32));
      z.part = std::max(z.part, (int64_t)atb_chunks(s.m, c, c) * c * c);
      if (P.alg4) {
        z.U = std::max(z.U, s.m * (int64_t)c);
        z.part = std::max(z.part, (int64_t)atb_chunks(s.n, c, c) * c * c);
      }
    }
    // with eps the run-time n may fall to <= kGramMax and take the Gram path
    // (atb_chunks(m, n, c) * n <= 1024 * 64 for every n, so 65536 * kCMax covers any
    // shape a prescribed-accuracy step can take)
    if (!P.fixed) z.part = std::max<int64_t>(z.part, (int64_t)65536 * kCMax);
    z.part = std::max<int64_t>(z.part, 2 * 8192);   // two per-workgroup sums of k_ax (<= 8192 groups each)
  }
  return z;
}

size_t layout_work(const Sizes& z, int d, char* base, Work* w) {
  size_t off = 0;
  auto take = [&](size_t nbytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(nbytes);
    return p;
  };
  Work tmp;
  Work& W = w ? *w : tmp;
  W.carry[0] = (double*)take(z.carry * 8);
  W.carry[1] = (double*)take(z.carry * 8);
  W.Y = (double*)take(z.Y * 8);
  W.U = (double*)take(z.U * 8);
  W.X = (double*)take(z.X * 8);
  W.M = (double*)take(z.X * 8);
  W.part = (double*)take(z.part * 8);
  W.part_len = z.part;
  W.H = (double*)take((size_t)kCMax * kCMax * 8);
  W.K = (double*)take((size_t)kCMax * kCMax * 8);
  W.V1 = (double*)take(z.V1 * 8);
  W.W = (double*)take((size_t)kCMax * kCMax * 8);
  W.normA2 = (double*)take(64);
  W.cpart = (double*)take((size_t)kCarryParts * 8);
  W.fold = (double*)take(z.fold * 8);
  W.fold_len = z.fold;
  W.recs = (StepRec*)take(sizeof(StepRec) * (size_t)d);
  W.dstate = (DeflState*)take(sizeof(DeflState));
  W.bytes = off;
  return off;
}

int check_limits(const Problem& P, const std::vector<Step>& S) {
  for (const Step& s : S) {
    if (P.variant == TT_SVD && P.fixed && s.r > TT_MAX_ELL)
      return fail(TT_EUNSUPPORTED, "TT-SVD step for core %d asks for rank %d > %d", s.core, s.r, TT_MAX_ELL);
    if (P.defl) {
      if (P.fixed && s.r > TT_MAX_ELL)
        return fail(TT_EUNSUPPORTED, "step for core %d asks for rank %d > %d", s.core, s.r, TT_MAX_ELL);
      if (s.n > kGramMax && s.n > kDeflMaxN)
        return fail(TT_EUNSUPPORTED, "deflation step for core %d: core side n = %d > %d", s.core, s.n, kDeflMaxN);
      continue;
    }
    const int ell = P.fixed ? step_ell(P, s, 0) : std::min<int64_t>(TT_MAX_ELL, std::min<int64_t>(s.n, s.m));
    if (P.fixed && ell > TT_MAX_ELL)
      return fail(TT_EUNSUPPORTED, "step for core %d needs ell = %d > %d (n = %d, m = %lld)", s.core,
                  ell, TT_MAX_ELL, s.n, (long long)s.m);
    if (s.n > (1 << 20)) return fail(TT_EUNSUPPORTED, "core side n = %d too large", s.n);
  }
  return TT_OK;
}

// ---- one step --------------------------------------------------------------
struct StepIO {
  const void* A;
  int a_f32;
  void* out;         // carry (next A) or the last core
  int out_f32;       // carry stored in FP32 (mixed precision, not the last core)
  double* core;      // core buffer of this step
};

// X = orth(M) for an iterate of the power loop: the option's orthonormaliser
// for the intermediate ones, Householder QR for the last (which feeds the
// Rayleigh-Ritz step)
hipError_t orth_iterate(const Problem& P, bool intermediate, double* M, double* X, int n, int c, const Work& W,
                        hipStream_t st) {
  if (intermediate && P.o.orth == TT_ORTH_CHOLQR && c <= n)
    return launch_orth_cholqr(M, X, n, c, W.part, W.part_len, st);
  return launch_orth(M, X, n, c, W.part, W.part_len, st);
}

// The fields of a step's solve arguments that define its test matrix.
SolveArgs sketch_args(const Problem& P, const Step& s, int ell) {
  SolveArgs a{};
  a.n = s.n;
  a.ell = ell;
  a.q = P.o.q;
  a.seed = P.o.seed;
  a.label = s.core;
  a.n_mode = s.n_mode;
  a.n_rank = s.n_rank;
  a.mode_fastest = s.mode_fastest;
  return a;
}

// sketch_ready: the previous carry pass already wrote this step's test matrix
// to W.X and the first product A X to W.Y (used unless this is a retry with a
// wider sketch)
int run_step_defl(const Problem& P, const Step& s, int cap, const SolveArgs& a, bool first, const StepIO& io,
                  StepRec* prev, int prev_parts, const Work& W, hipStream_t st, Prof& PF);

int run_step(const Problem& P, const Step& s, int ell, int si, bool first, const StepIO& io,
             StepRec* prev, int prev_parts, const Work& W, hipStream_t st, Prof& PF, bool retry,
             bool sketch_ready = false) {
  SolveArgs a = sketch_args(P, s, ell);
  a.r_fixed = P.fixed ? s.r : 0;
  const double wk = P.fixed ? 0.0 : P.w[s.unfolding - 1];
  a.eps_factor2 = wk * P.eps_rule * wk * P.eps_rule;
  a.max_rank = P.fixed ? 0 : (int)std::min<int64_t>(s.r, TT_MAX_ELL);
  a.core_layout = (P.sweep == TT_L2R) ? 0 : 1;
  a.core = io.core;
  a.V1 = W.V1;
  a.W = W.W;
  a.rec = W.recs + si;
  a.normA2 = W.normA2;
  a.first = first ? 1 : 0;
  a.normC2_src = first ? nullptr : &prev->carry2;
  if (!first && prev_parts > 0) {
    // the previous carry's sum of squares is still in partials: the solve reduces it
    a.nc_parts = W.cpart;
    a.nc_n = prev_parts;
    a.nc_out = &prev->carry2;
  }
  const int64_t m = s.m;
  const int n = s.n;
  StepRec* rec = W.recs + si;

  const double sa = io.a_f32 ? 4.0 : 8.0;
  const double mn = (double)m * n;
  if (P.defl) return run_step_defl(P, s, ell, a, first, io, prev, prev_parts, W, st, PF);
  if (step_gram(P, s)) {
    // H = A^T A in one pass, then everything else on n x n (a retry with a wider
    // sketch reuses H: it does not depend on ell)
    if (!retry) {
      const int nch = atb_chunks(m, n, n);
      LAUNCH(PF, KC_ATB, mn * sa + (double)n * n * 8, 2.0 * mn * n,
             launch_atb(io.A, io.a_f32, io.A, io.a_f32, m, n, n, s.layout, W.part, nch, st));
      LAUNCH(PF, KC_REDUCE, (double)(nch + 1) * n * n * 8, (double)nch * n * n,
             launch_reduce(W.part, nch, (int64_t)n * n, W.H, nullptr, st));
    }
    LAUNCH(PF, KC_SMALL, 0, 0, launch_gram_solve(W.H, a, st));
  } else if (!P.alg4) {
    // sketch and q+1 power steps: X <- orth(A^T (A X)), starting from X = G
    const int c = ell;
    const int ach = ax_chunks(m, n, c);
    const double mc = (double)m * c;
    const bool have_y = sketch_ready && !retry;
    if (!have_y) LAUNCH(PF, KC_SMALL, 0, 0, launch_gen_sketch(W.X, a, st));
    const int qp = power_steps(P);
    for (int it = 0; it <= qp; ++it) {
      if (P.mixed) {
        // mixed precision: power products on FP32 (or BF16) operands with FP32
        // accumulation, FP32 iterate
        if (!(have_y && it == 0))
          LAUNCH(PF, KC_AX, mn * sa + mc * 4 + (double)n * c * 8, 2.0 * mn * c,
                 launch_ax_lp(io.A, io.a_f32, W.X, (float*)W.Y, m, n, c, s.layout, P.bf16, st));
        const int nch = atb_lp_chunks(m, n);
        double* dst = nch == 1 ? W.M : W.part;   // a single chunk is the sum itself
        if (P.bf16)
          LAUNCH(PF, KC_ATB, mn * sa + mc * 4 + (double)n * c * 8, 2.0 * mn * c,
                 launch_atb_lp(io.A, io.a_f32, (const float*)W.Y, m, n, c, s.layout, dst, nch, 1, st));
        else
          LAUNCH(PF, KC_ATB, mn * sa + mc * 4 + (double)n * c * 8, 2.0 * mn * c,
                 launch_atb2(io.A, io.a_f32, W.Y, 1, m, n, c, s.layout, io.a_f32, dst, nch, st));
        if (nch > 1)
          LAUNCH(PF, KC_REDUCE, (double)(nch + 1) * n * c * 8, (double)nch * n * c,
                 launch_reduce(W.part, nch, (int64_t)n * c, W.M, nullptr, st));
      } else if (P.o.fuse_ata && !(first && it == 0) && fused_ata_ok(io.a_f32, m, n, c, s.layout)) {
        const int fb = fused_ata_blocks(m);
        LAUNCH(PF, KC_ATA, mn * sa + (double)n * c * 8 + (double)fb * n * c * 8, 4.0 * mn * c,
               launch_fused_ata((const double*)io.A, W.X, m, n, c, W.part, fb, st));
        LAUNCH(PF, KC_REDUCE, (double)(fb + 1) * n * c * 8, (double)fb * n * c,
               launch_reduce(W.part, fb, (int64_t)n * c, W.M, nullptr, st));
      } else {
        if (!(have_y && it == 0))
          LAUNCH(PF, KC_AX, mn * sa + mc * 8 + (double)n * c * 8, 2.0 * mn * c,
                 launch_ax(io.A, io.a_f32, W.X, W.Y, 0, m, n, c, s.layout, ach,
                           (first && it == 0) ? W.part : nullptr, nullptr, nullptr, st));
        if (first && it == 0)
          LAUNCH(PF, KC_REDUCE, (double)ach * 8, ach, launch_reduce(W.part, ach, 1, W.normA2, nullptr, st));
        // a single chunk is the sum itself: written straight to M, no reduction
        const int nch = atb2_chunks(m, n);
        LAUNCH(PF, KC_ATB, mn * sa + mc * 8 + (double)n * c * 8, 2.0 * mn * c,
               launch_atb2(io.A, io.a_f32, W.Y, 0, m, n, c, s.layout, 0, nch == 1 ? W.M : W.part, nch, st));
        if (nch > 1)
          LAUNCH(PF, KC_REDUCE, (double)(nch + 1) * n * c * 8, (double)nch * n * c,
                 launch_reduce(W.part, nch, (int64_t)n * c, W.M, nullptr, st));
      }
      LAUNCH(PF, KC_SMALL, 0, 0, orth_iterate(P, it < qp, W.M, W.X, n, c, W, st));
    }
    // Rayleigh-Ritz: Y = A X, K = Y^T Y
    // the Rayleigh-Ritz pass keeps Y in FP64 (its Gram decides the rank); in the
    // mixed form it is also the pass that measures ||A||^2 on the first step
    const bool rr_norm = first && P.mixed;
    LAUNCH(PF, KC_AX, mn * sa + mc * 8 + (double)n * c * 8, 2.0 * mn * c,
           launch_ax(io.A, io.a_f32, W.X, W.Y, 0, m, n, c, s.layout, ach, rr_norm ? W.part : nullptr, nullptr,
                     nullptr, st));
    if (rr_norm) LAUNCH(PF, KC_REDUCE, (double)ach * 8, ach, launch_reduce(W.part, ach, 1, W.normA2, nullptr, st));
    const int kch = atb_chunks(m, c, c);
    LAUNCH(PF, KC_GRAM_Y, mc * 8 + (double)c * c * 8, 2.0 * mc * c,
           launch_atb(W.Y, 0, W.Y, 0, m, c, c, s.layout, kch == 1 ? W.K : W.part, kch, st));
    if (kch > 1)
      LAUNCH(PF, KC_REDUCE, (double)(kch + 1) * c * c * 8, (double)kch * c * c,
             launch_reduce(W.part, kch, (int64_t)c * c, W.K, nullptr, st));
    if (first) a.normC2_src = W.normA2;
    LAUNCH(PF, KC_SMALL, 0, 0, launch_rr_solve(W.K, W.X, a, st));
  } else {
    // Alg. 4: X spans (A^T A)^q G, Y = A X spans the range sketch (A A^T)^q A G
    const int c = ell;
    const int ach = ax_chunks(m, n, c);
    const double mc = (double)m * c;
    bool need_norm = first;
    LAUNCH(PF, KC_SMALL, 0, 0, launch_gen_sketch(W.X, a, st));
    for (int it = 0; it < P.o.q; ++it) {
      if (!P.mixed && !need_norm && P.o.fuse_ata && fused_ata_ok(io.a_f32, m, n, c, s.layout)) {
        const int fb = fused_ata_blocks(m);
        LAUNCH(PF, KC_ATA, mn * sa + (double)n * c * 8 + (double)fb * n * c * 8, 4.0 * mn * c,
               launch_fused_ata((const double*)io.A, W.X, m, n, c, W.part, fb, st));
        LAUNCH(PF, KC_REDUCE, (double)(fb + 1) * n * c * 8, (double)fb * n * c,
               launch_reduce(W.part, fb, (int64_t)n * c, W.M, nullptr, st));
        LAUNCH(PF, KC_SMALL, 0, 0, orth_iterate(P, it + 1 < P.o.q, W.M, W.X, n, c, W, st));
        continue;
      }
      const double sy = P.mixed ? 4.0 : 8.0;
      LAUNCH(PF, KC_AX, mn * sa + mc * sy + (double)n * c * 8, 2.0 * mn * c,
             launch_ax(io.A, io.a_f32, W.X, W.Y, P.mixed, m, n, c, s.layout, ach,
                       need_norm ? W.part : nullptr, nullptr, nullptr, st));
      if (need_norm) {
        LAUNCH(PF, KC_REDUCE, (double)ach * 8, ach, launch_reduce(W.part, ach, 1, W.normA2, nullptr, st));
        need_norm = false;
      }
      const int nch = atb2_chunks(m, n);
      LAUNCH(PF, KC_ATB, mn * sa + mc * sy + (double)n * c * 8, 2.0 * mn * c,
             launch_atb2(io.A, io.a_f32, W.Y, P.mixed, m, n, c, s.layout, 0, W.part, nch, st));
      LAUNCH(PF, KC_REDUCE, (double)(nch + 1) * n * c * 8, (double)nch * n * c,
             launch_reduce(W.part, nch, (int64_t)n * c, W.M, nullptr, st));
      LAUNCH(PF, KC_SMALL, 0, 0, orth_iterate(P, it + 1 < P.o.q, W.M, W.X, n, c, W, st));
    }
    LAUNCH(PF, KC_AX, mn * sa + mc * 8 + (double)n * c * 8, 2.0 * mn * c,
           launch_ax(io.A, io.a_f32, W.X, W.Y, 0, m, n, c, s.layout, ach,
                     need_norm ? W.part : nullptr, nullptr, nullptr, st));
    if (need_norm) LAUNCH(PF, KC_REDUCE, (double)ach * 8, ach, launch_reduce(W.part, ach, 1, W.normA2, nullptr, st));
    // U = orth(Y): two eigen-based Cholesky-QR rounds, Y -> U (round 1) -> Y (round 2)
    const int kch = atb_chunks(m, c, c);
    const int ych = ax_chunks(m, c, c);
    for (int round = 0; round < 2; ++round) {
      double* src = round == 0 ? W.Y : W.U;
      double* dst = round == 0 ? W.U : W.Y;
      LAUNCH(PF, KC_GRAM_Y, mc * 8 + (double)c * c * 8, 2.0 * mc * c,
             launch_atb(src, 0, src, 0, m, c, c, s.layout, W.part, kch, st));
      LAUNCH(PF, KC_REDUCE, (double)(kch + 1) * c * c * 8, (double)kch * c * c,
             launch_reduce(W.part, kch, (int64_t)c * c, W.K, nullptr, st));
      LAUNCH(PF, KC_SMALL, 0, 0, launch_alg4_basis(W.K, W.H, c, st));
      LAUNCH(PF, KC_GRAM_Y, 2.0 * mc * 8 + (double)c * c * 8, 2.0 * mc * c,
             launch_ax(src, 0, W.H, dst, 0, m, c, c, s.layout, ych, nullptr, nullptr, nullptr, st));
    }
    // Bt = A^T U (n x ell), E = Bt^T Bt
    const int nch = atb2_chunks(m, n);
    LAUNCH(PF, KC_ATB, mn * sa + mc * 8 + (double)n * c * 8, 2.0 * mn * c,
           launch_atb2(io.A, io.a_f32, W.Y, 0, m, n, c, s.layout, 0, W.part, nch, st));
    LAUNCH(PF, KC_REDUCE, (double)(nch + 1) * n * c * 8, (double)nch * n * c,
           launch_reduce(W.part, nch, (int64_t)n * c, W.M, nullptr, st));
    const int ech = atb_chunks(n, c, c);
    LAUNCH(PF, KC_SMALL, 0, 0, launch_atb(W.M, 0, W.M, 0, n, c, c, COL, W.part, ech, st));
    LAUNCH(PF, KC_REDUCE, (double)(ech + 1) * c * c * 8, (double)ech * c * c,
           launch_reduce(W.part, ech, (int64_t)c * c, W.K, nullptr, st));
    if (first) a.normC2_src = W.normA2;
    LAUNCH(PF, KC_SMALL, 0, 0, launch_alg4_solve(W.K, W.M, a, st));
  }
  return TT_OK;
}

// One step with the deflation inner kernel.  n <= kGramMax: H = A^T A in one
// pass and the whole search on H in one workgroup.  Otherwise one pass over A
// per power step, each followed by the fixed-order reduction of its partials
// and a one-workgroup update (projection, normalisation, bookkeeping); the pass
// of vector j's first power step also measures the energy of vector j - 1, and
// a last pass that of the final vector.  With a prescribed accuracy the host
// reads the search state after every vector and stops launching once the rank
// rule is met (later launches of a finished search would do nothing).
// ||C||^2 of the step is measured on A itself (trace of H, or the first pass).
int run_step_defl(const Problem& P, const Step& s, int cap, const SolveArgs& a, bool first, const StepIO& io,
                  StepRec* prev, int prev_parts, const Work& W, hipStream_t st, Prof& PF) {
  const int64_t m = s.m;
  const int n = s.n;
  const double sa = io.a_f32 ? 4.0 : 8.0;
  const double mn = (double)m * n;
  SolveArgs b = a;
  b.nc_parts = nullptr;
  b.nc_n = 0;
  b.nc_out = nullptr;
  if (!first && prev_parts > 0)   // the previous carry's ||.||^2 is still in partials
    LAUNCH(PF, KC_REDUCE, (double)prev_parts * 8, prev_parts,
           launch_reduce(W.cpart, prev_parts, 1, &prev->carry2, nullptr, st));
  if (step_gram(P, s)) {
    const int nch = atb_chunks(m, n, n);
    LAUNCH(PF, KC_ATB, mn * sa + (double)n * n * 8, 2.0 * mn * n,
           launch_atb(io.A, io.a_f32, io.A, io.a_f32, m, n, n, s.layout, W.part, nch, st));
    LAUNCH(PF, KC_REDUCE, (double)(nch + 1) * n * n * 8, (double)nch * n * n,
           launch_reduce(W.part, nch, (int64_t)n * n, W.H, nullptr, st));
    LAUNCH(PF, KC_SMALL, 0, 0, launch_defl_gram(W.H, b, cap, st));
    return TT_OK;
  }
  DeflArgs D;
  D.a = b;
  D.cap = cap;
  D.V = W.X;
  D.x = W.X + (int64_t)n * cap;
  D.st = W.dstate;
  const int ng = defl_pass_groups(m, n, s.layout);
  double* stripes = W.part + (int64_t)ng * (n + 3);   // after the pass partials (sized for both)
  if ((int64_t)(ng + kReduceStripes) * (n + 3) > W.part_len)
    return fail(TT_EINVAL, "internal: deflation scratch %lld doubles > %lld", (long long)(ng + kReduceStripes) * (n + 3),
                (long long)W.part_len);
  const double pb = mn * sa + (double)ng * (n + 3) * 8;   // A once, the partials written
  LAUNCH(PF, KC_SMALL, 0, 0, launch_defl_start(D, st));
  bool done = false;
  for (int j = 0; j < cap && !done; ++j) {
    for (int it = 0; it < P.o.q; ++it) {
      const bool hw = (it == 0 && j > 0), fp = (j == 0 && it == 0);
      LAUNCH(PF, KC_DEFL, pb + (hw ? 2.0 : 1.0) * n * 8, (hw ? 6.0 : 4.0) * mn,
             launch_defl_pass(io.A, io.a_f32, m, n, s.layout, D.x, hw ? D.V + (int64_t)(j - 1) * n : nullptr,
                              fp ? 1 : 0, W.part, ng, st));
      LAUNCH(PF, KC_REDUCE, (double)(ng + 1) * (n + 3) * 8, (double)ng * (n + 3),
             launch_reduce(W.part, ng, (int64_t)n + 3, W.M, nullptr, st, stripes));
      LAUNCH(PF, KC_SMALL, 0, 0, launch_defl_update(W.M, D, j, hw ? 1 : 0, it == P.o.q - 1 ? 1 : 0, fp ? 1 : 0, st));
    }
    if (!P.fixed) {
      DeflState hs;
      HIP_OK(hipMemcpyAsync(&hs, W.dstate, sizeof(hs), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      done = hs.done != 0 || !std::isfinite(hs.normC2);   // a non-finite input stops the search
    }
  }
  if (!done) {
    // the energy of the last vector
    LAUNCH(PF, KC_DEFL, pb + (double)n * 8, 2.0 * mn,
           launch_defl_pass(io.A, io.a_f32, m, n, s.layout, nullptr, D.V + (int64_t)(cap - 1) * n, 0, W.part, ng,
                            st));
    LAUNCH(PF, KC_REDUCE, (double)(ng + 1) * (n + 3) * 8, (double)ng * (n + 3),
           launch_reduce(W.part, ng, (int64_t)n + 3, W.M, nullptr, st, stripes));
    LAUNCH(PF, KC_SMALL, 0, 0, launch_defl_last(W.M, D, st));
  }
  LAUNCH(PF, KC_SMALL, 0, 0, launch_defl_finish(D, st));
  return TT_OK;
}

// defer_norm: leave ||carry||^2 as per-workgroup partials in W.cpart for the
// next step's solve to reduce (*parts_out = their count, else 0).
// The next step's first sketch product formed in this step's carry pass (see
// tt_carry_sketch.hip): its slab height m2, slab count I (= the next mode's
// extent), sketch width c and element size of Y.
struct NextSketch {
  bool on = false;
  int64_t m2 = 0;
  int I = 0, c = 0;
  double sy = 8.0;
};

int carry_step(const Problem& P, const Step& s, int ell, int r, const StepIO& io, const Work& W,
               StepRec* rec, hipStream_t st, Prof& PF, bool defer_norm, int* parts_out,
               const NextSketch& nx = NextSketch()) {
  const int64_t m = s.m;
  const bool direct = step_gram(P, s) || P.defl;   // carry = A V1 (else Y W from the Rayleigh-Ritz pass)
  const int ach = nx.on ? carry_sketch_groups(nx.m2, io.a_f32, io.out_f32)
                        : (direct ? ax_chunks(m, s.n, r) : ax_chunks(m, ell, r));
  const double sa = io.a_f32 ? 4.0 : 8.0;
  const double so = io.out_f32 ? 4.0 : 8.0;
  const double mr = (double)m * r;
  double* rerr = io.out_f32 ? W.part + 8192 : nullptr;
  const bool defer = defer_norm && ach <= kCarryParts;
  double* nparts = defer ? W.cpart : W.part;
  *parts_out = defer ? ach : 0;
  if (nx.on) {
    const double mn = (double)m * s.n;
    LAUNCH(PF, KC_CARRY, mn * sa + mr * so + (double)nx.m2 * nx.c * nx.sy + (double)nx.I * s.n * nx.c * 8,
           2.0 * mn * r + 2.0 * mn * nx.c,
           launch_carry_sketch(io.A, io.a_f32, nx.m2, nx.I, s.n, W.V1, r, W.fold, nx.c, io.out, io.out_f32, W.Y,
                               nparts, rerr, ach, st));
  } else if (direct) {
    const double mn = (double)m * s.n;
    LAUNCH(PF, KC_CARRY, mn * sa + mr * so + (double)s.n * r * 8, 2.0 * mn * r,
           launch_ax(io.A, io.a_f32, W.V1, io.out, io.out_f32, m, s.n, r, s.layout, ach, nullptr, nparts, rerr, st));
  } else {
    const double ml = (double)m * ell;
    LAUNCH(PF, KC_CARRY, ml * 8 + mr * so + (double)ell * r * 8, 2.0 * ml * r,
           launch_ax(W.Y, 0, W.W, io.out, io.out_f32, m, ell, r, s.layout, ach, nullptr, nparts, rerr, st));
  }
  if (!defer) LAUNCH(PF, KC_REDUCE, (double)ach * 8, ach, launch_reduce(W.part, ach, 1, &rec->carry2, nullptr, st));
  if (rerr) LAUNCH(PF, KC_REDUCE, (double)ach * 8, ach, launch_reduce(rerr, ach, 1, &rec->rho2, nullptr, st));
  if (P.o.exact_delta) {
    const int rch = resid_chunks(m);
    const double mn = (double)m * s.n;
    LAUNCH(PF, KC_RESID, mn * sa + mr * so, 2.0 * mn * r + 2.0 * mn,
           launch_resid(io.A, io.a_f32, io.out, io.out_f32, W.V1, m, s.n, r, s.layout, rch, W.part, st));
    LAUNCH(PF, KC_REDUCE, (double)rch * 8, rch, launch_reduce(W.part, rch, 1, &rec->resid2, nullptr, st));
  }
  return TT_OK;
}

}  // namespace

// ============================================================================
extern "C" {

void tt_default_opts(tt_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->q = 1;
  o->oversample = 8;
}

const char* tt_last_error(void) { return g_err; }

const char* tt_kernel_class_name(int c) { return (c >= 0 && c < TT_NKCLASS) ? kClassNames[c] : nullptr; }

int tt_utv_workspace(int d, const int64_t* dims, const int64_t* ranks, double eps, tt_sweep sweep,
                     tt_variant variant, tt_dtype dtype, const tt_opts* opts, size_t* bytes) {
  if (!bytes) return fail(TT_EINVAL, "bytes is NULL");
  Problem P;
  int rc = check_args(d, dims, ranks, eps, sweep, variant, dtype, opts, P);
  if (rc) return rc;
  std::vector<Step> S;
  plan_steps(P, P.ranks, S, nullptr);
  rc = check_limits(P, S);
  if (rc) return rc;
  *bytes = layout_work(size_bounds(P, S), d, nullptr, nullptr);
  return TT_OK;
}

int tt_utv_core_capacity(int d, const int64_t* dims, const int64_t* ranks, double eps,
                         const tt_opts* opts, int64_t* capacity) {
  if (!capacity) return fail(TT_EINVAL, "capacity is NULL");
  Problem P;
  int rc = check_args(d, dims, ranks, eps, TT_L2R, TT_ULV, TT_F64, opts, P);
  if (rc) return rc;
  // the largest rank each bond can take in either sweep direction
  int64_t r[TT_MAX_D + 1];
  for (int k = 0; k <= d; ++k) {
    const int64_t left = prod(P.dims, 0, k), right = prod(P.dims, k, d);
    int64_t b = std::min(left, right);
    if (k > 0 && k < d) b = std::min(b, P.ranks[k]);
    r[k] = (k == 0 || k == d) ? 1 : b;
  }
  for (int k = 0; k < d; ++k) capacity[k] = r[k] * P.dims[k] * r[k + 1];
  return TT_OK;
}

int tt_utv_decompose(const void* A, tt_dtype dtype, int d, const int64_t* dims, const int64_t* ranks,
                     double eps, tt_sweep sweep, tt_variant variant, const tt_opts* opts,
                     void* work, size_t work_bytes, double* const* cores, tt_report* rep,
                     void* stream) {
  Problem P;
  int rc = check_args(d, dims, ranks, eps, sweep, variant, dtype, opts, P);
  if (rc) return rc;
  if (!A) return fail(TT_EINVAL, "A is NULL");
  if (!cores) return fail(TT_EINVAL, "cores is NULL");
  for (int k = 0; k < d; ++k)
    if (!cores[k]) return fail(TT_EINVAL, "cores[%d] is NULL", k);
  std::vector<Step> S;
  plan_steps(P, P.ranks, S, nullptr);
  rc = check_limits(P, S);
  if (rc) return rc;
  Work W;
  const size_t need = layout_work(size_bounds(P, S), d, (char*)work, &W);
  if (!work || work_bytes < need)
    return fail(TT_ENOSPC, "workspace %zu bytes < %zu needed", work_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  Prof PF;
  PF.on = P.o.profile != 0;
  PF.mask = P.o.profile;
  PF.st = st;
  // fixed ranks and no report: the call only enqueues kernels and never waits
  // on the stream (so it can be recorded into a graph); a non-finite input is
  // then not caught after the first pass and leaves non-finite cores
  const bool enqueue_only = P.fixed && !rep && !PF.on;

  const int nsteps = d - 1;
  int64_t r_run[TT_MAX_D + 1];
  for (int k = 0; k <= d; ++k) r_run[k] = P.ranks[k];
  std::vector<int> ells(nsteps, 0), rs(nsteps, 0);
  const void* curA = A;
  int a_f32 = (dtype == TT_F32);
  int prev_r = 0;
  int prev_parts = 0;   // partials of the previous carry's ||.||^2 left for this step's solve
  bool sketch_ready = false;   // the previous carry pass formed this step's first sketch product
  bool all_sat = true;
  std::vector<StepRec> host(nsteps);
  for (int si = 0; si < nsteps; ++si) {
    // shape of this step from the ranks decided so far
    std::vector<Step> S2;
    plan_steps(P, r_run, S2, nullptr);
    Step s = S2[si];
    const bool first = (si == 0);
    const bool last = (si == nsteps - 1);
    StepIO io;
    io.A = curA;
    io.a_f32 = a_f32;
    io.core = cores[s.core - 1];
    const int final_core = (P.sweep == TT_L2R) ? d - 1 : 0;
    io.out = last ? (void*)cores[final_core] : (void*)W.carry[si & 1];
    io.out_f32 = (P.mixed && !last) ? 1 : 0;
    int ell = step_ell(P, s, first ? 2 * P.o.oversample : prev_r + P.o.oversample);
    if (ell < 1) ell = 1;
    if (ell > TT_MAX_ELL) ell = TT_MAX_ELL;
    int r;
    bool retry = false;
    while (true) {
      rc = run_step(P, s, ell, si, first, io, si > 0 ? W.recs + (si - 1) : nullptr, prev_parts, W, st, PF, retry,
                    sketch_ready);
      if (rc) return rc;
      // ||A||^2 is known after the first pass over A: a non-finite input stops
      // the sweep here instead of running every step on NaNs
      if (first && !retry && !enqueue_only) {
        double nA2_first = 0.0;
        HIP_OK(hipMemcpyAsync(&nA2_first, W.normA2, sizeof(double), hipMemcpyDeviceToHost, st));
        if (!P.fixed) HIP_OK(hipMemcpyAsync(&host[si], W.recs + si, sizeof(StepRec), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (!isfinite(nA2_first)) {
          if (rep) {
            memset(rep, 0, sizeof(*rep));
            rep->d = d;
            rep->norm_A = nA2_first;
          }
          return fail(TT_ENONFINITE, "input holds non-finite values (||A||^2 = %g after the first pass)", nA2_first);
        }
      }
      const bool synced = first && !retry;
      retry = true;
      if (P.fixed) { r = std::min(s.r, ell); break; }
      if (!synced) {
        HIP_OK(hipMemcpyAsync(&host[si], W.recs + si, sizeof(StepRec), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
      }
      r = host[si].r;
      const int lim = (int)std::min<int64_t>(std::min<int64_t>(s.n, s.m), TT_MAX_ELL);
      if (host[si].sat || ell >= lim || (s.r > 0 && r >= s.r)) {
        if (!host[si].sat) all_sat = false;
        break;
      }
      ell = std::min(2 * ell, lim);
    }
    // Right to left, a Gram-mode step before a sketched one: the carry pass also
    // forms the next step's first sketch product (its test matrix is drawn now,
    // with the width the next step will start from)
    NextSketch nx;
    if (!last && P.sweep == TT_R2L && !P.alg4 && !P.defl && !P.o.separate_sketch && !P.bf16 && step_gram(P, s)) {
      int64_t r_next[TT_MAX_D + 1];
      for (int k = 0; k <= d; ++k) r_next[k] = r_run[k];
      r_next[s.core - 1] = r;
      std::vector<Step> S3;
      plan_steps(P, r_next, S3, nullptr);
      const Step& s2 = S3[si + 1];
      int ell2 = step_ell(P, s2, r + P.o.oversample);
      ell2 = std::max(1, std::min(ell2, TT_MAX_ELL));
      const int I = s2.n_mode;
      const bool ata = P.o.fuse_ata && fused_ata_ok(io.out_f32, s2.m, s2.n, ell2, s2.layout);
      if (!step_gram(P, s2) && !ata && s2.m * I == s.m && (int64_t)s2.n == (int64_t)I * r &&
          W.fold_len >= (int64_t)I * s.n * ell2 &&
          carry_sketch_ok(io.A, io.a_f32, io.out, io.out_f32, W.Y, s2.m, I, s.n, r, ell2)) {
        const SolveArgs a2 = sketch_args(P, s2, ell2);
        LAUNCH(PF, KC_SMALL, 0, 0, launch_gen_sketch(W.X, a2, st));
        LAUNCH(PF, KC_SMALL, 0, 0, launch_sketch_fold(W.V1, W.X, W.fold, I, s.n, r, ell2, st));
        nx.on = true;
        nx.m2 = s2.m;
        nx.I = I;
        nx.c = ell2;
        nx.sy = io.out_f32 ? 4.0 : 8.0;
      }
    }
    // the last carry's norm is reduced at once (no later solve reads it)
    rc = carry_step(P, s, ell, r, io, W, W.recs + si, st, PF, !last, &prev_parts, nx);
    if (rc) return rc;
    sketch_ready = nx.on;
    ells[si] = P.defl ? r : ell;
    rs[si] = r;
    // rank of the bond this step decided
    if (P.sweep == TT_L2R) r_run[s.core] = r; else r_run[s.core - 1] = r;
    prev_r = r;
    curA = io.out;
    a_f32 = io.out_f32;
  }
  if (enqueue_only) return TT_OK;
  HIP_OK(hipMemcpyAsync(host.data(), W.recs, sizeof(StepRec) * nsteps, hipMemcpyDeviceToHost, st));
  double nA2 = 0.0;
  HIP_OK(hipMemcpyAsync(&nA2, W.normA2, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  // the bound the report states; in eps mode it must not exceed eps ||A||.
  // Checked only when the step errors are measured (exact_delta): the default
  // estimates sqrt(||C||^2 - ||carry||^2) carry rounding noise of about
  // 1e-13 ||C||^2 in delta^2, which at eps ~ 1e-6 is as large as the
  // a-priori FP32 carry budget the rank rule already set aside.
  if (P.o.exact_delta) {
    double sum2 = 0.0, sum1 = 0.0, rho_sum = 0.0;
    for (int si = 0; si < nsteps; ++si) {
      const StepRec& h = host[si];
      double dl2 = (h.resid2 >= 0.0) ? h.resid2 : h.normC2 - h.carry2;
      if (dl2 < 0.0) dl2 = 0.0;
      sum2 += dl2;
      sum1 += sqrt(dl2);
      rho_sum += sqrt(std::max(h.rho2, 0.0));
    }
    const double bound = (P.alg4 ? sum1 : sqrt(sum2)) + rho_sum;
    if (!P.fixed && !(bound <= P.eps * sqrt(std::max(nA2, 0.0)))) all_sat = false;
  }
  if (rep) {
    memset(rep, 0, sizeof(*rep));
    rep->d = d;
    for (int k = 0; k <= d; ++k) rep->ranks[k] = r_run[k];
    rep->ranks[0] = rep->ranks[d] = 1;
    double sum2 = 0.0, sum1 = 0.0, rho_sum = 0.0;
    std::vector<Step> S2;
    plan_steps(P, r_run, S2, nullptr);
    for (int si = 0; si < nsteps; ++si) {
      const int u = S2[si].unfolding - 1;
      const StepRec& h = host[si];
      double dl2 = (h.resid2 >= 0.0) ? h.resid2 : h.normC2 - h.carry2;
      if (dl2 < 0.0) dl2 = 0.0;
      rep->delta[u] = sqrt(dl2);
      rep->normC[u] = sqrt(std::max(h.normC2, 0.0));
      rep->ell[u] = ells[si];
      rep->sweeps[u] = h.sweeps;
      rep->rho[u] = sqrt(std::max(h.rho2, 0.0));
      rho_sum += rep->rho[u];
      sum2 += dl2;
      sum1 += sqrt(dl2);
      if (!P.fixed && !h.sat) all_sat = false;
    }
    rep->norm_A = sqrt(std::max(nA2, 0.0));
    for (const Prof::Rec& pr : PF.recs) {
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, pr.a, pr.b));
      tt_kstat& k = rep->kstat[pr.cls];
      k.launches += 1;
      k.ms += ms;
      k.bytes += pr.bytes;
      k.flops += pr.flops;
    }
    // storing a carry in FP32 perturbs the matrix the rest of the sweep
    // factorises by rho_k; the later steps are norm-non-increasing, so the
    // perturbations add to the bound of the exact sweep
    rep->err_bound = (P.alg4 ? sum1 : sqrt(sum2)) + rho_sum;
    rep->err_bound_measured = P.o.exact_delta ? 1 : 0;
    rep->rank_rule_met = P.fixed ? 1 : (all_sat ? 1 : 0);
  }
  if (!isfinite(nA2)) return fail(TT_ENONFINITE, "input holds non-finite values (||A||^2 = %g)", nA2);
  if (!P.fixed && !all_sat)
    return fail(TT_ERANK, "eps = %g not reached within the rank cap", P.eps);
  return TT_OK;
}

}  // extern "C"

namespace {

// Workspace of tt_utv_decompose_noalloc: one array per device, held from the
// library's load to the end of the process.  Its name is a host-side stand-in;
// kernels get the device address that hipGetSymbolAddress returns for the
// current device (looked up once per device, on the first call there).
static __device__ __align__(256) double scratch[TT_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_of_current_device(void** ptr) {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TT_EUNSUPPORTED, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(TT_EHIP, "hipGetSymbolAddress returned a null scratch address on device %d", dev);
    g_scratch_dev[dev] = p;
  }
  *ptr = g_scratch_dev[dev];
  return TT_OK;
}

}  // namespace

extern "C" {

int tt_utv_decompose_noalloc(const void* A, tt_dtype dtype, int d, const int64_t* dims, const int64_t* ranks,
                             double eps, tt_sweep sweep, tt_variant variant, const tt_opts* opts,
                             double* const* cores, tt_report* rep, void* stream) {
  size_t need = 0;
  int rc = tt_utv_workspace(d, dims, ranks, eps, sweep, variant, dtype, opts, &need);
  if (rc) return rc;
  if (need > (size_t)TT_NOALLOC_SCRATCH_BYTES)
    return fail(TT_ENOSPC, "problem needs %zu bytes of workspace, above the %zu-byte static scratch of "
                "tt_utv_decompose_noalloc (use tt_utv_decompose with a caller workspace)",
                need, (size_t)TT_NOALLOC_SCRATCH_BYTES);
  if (opts && opts->profile)
    return fail(TT_EINVAL, "opts.profile needs HIP events, which tt_utv_decompose_noalloc does not create");
  void* work = nullptr;
  rc = scratch_of_current_device(&work);
  if (rc) return rc;
  return tt_utv_decompose(A, dtype, d, dims, ranks, eps, sweep, variant, opts, work,
                          (size_t)TT_NOALLOC_SCRATCH_BYTES, cores, rep, stream);
}

}  // extern "C"

namespace {

// Reconstruction plan: split the train after core h so that the two partial
// products L (P_left x r_h) and R (r_h x P_right) are about equally long; the
// dense tensor is then one small-K GEMM L R (column-major = ivec order).
struct RecPlan {
  int h;
  int64_t left_max, right_max;
};

int rec_plan(int d, const int64_t* dims, const int64_t* ranks, RecPlan& rp) {
  if (d < 2 || d > TT_MAX_D || !dims || !ranks) return fail(TT_EINVAL, "bad train description");
  if (ranks[0] != 1 || ranks[d] != 1) return fail(TT_EINVAL, "r_0 and r_d must be 1");
  for (int k = 0; k < d; ++k)
    if (dims[k] < 1) return fail(TT_EINVAL, "dims[%d] < 1", k);
  for (int k = 0; k <= d; ++k)
    if (ranks[k] < 1 || ranks[k] > kCMax) return fail(TT_EUNSUPPORTED, "rank %lld outside [1, 64]", (long long)ranks[k]);
  double best = 1e300;
  rp.h = 1;
  for (int h = 1; h < d; ++h) {
    const double l = log((double)prod(dims, 0, h)), r = log((double)prod(dims, h, d));
    if (fabs(l - r) < best) { best = fabs(l - r); rp.h = h; }
  }
  rp.left_max = 1;
  for (int k = 2; k <= rp.h; ++k) rp.left_max = std::max(rp.left_max, prod(dims, 0, k) * ranks[k]);
  rp.right_max = 1;
  for (int k = d - 1; k >= rp.h + 1; --k) rp.right_max = std::max(rp.right_max, ranks[k - 1] * prod(dims, k - 1, d));
  return TT_OK;
}

}  // namespace

extern "C" {

int tt_reconstruct_workspace(int d, const int64_t* dims, const int64_t* ranks, size_t* bytes) {
  if (!bytes) return fail(TT_EINVAL, "bytes is NULL");
  RecPlan rp;
  int rc = rec_plan(d, dims, ranks, rp);
  if (rc) return rc;
  *bytes = 2 * align_up(rp.left_max * 8) + 2 * align_up(rp.right_max * 8);
  return TT_OK;
}

int tt_reconstruct(int d, const int64_t* dims, const int64_t* ranks, const double* const* cores,
                   void* out, tt_dtype dtype, void* work, size_t work_bytes, void* stream) {
  RecPlan rp;
  int rc = rec_plan(d, dims, ranks, rp);
  if (rc) return rc;
  if (!cores || !out) return fail(TT_EINVAL, "cores/out is NULL");
  if (dtype != TT_F64 && dtype != TT_F32) return fail(TT_EINVAL, "bad dtype");
  for (int k = 0; k < d; ++k)
    if (!cores[k]) return fail(TT_EINVAL, "cores[%d] is NULL", k);
  const size_t need = 2 * align_up(rp.left_max * 8) + 2 * align_up(rp.right_max * 8);
  if (work_bytes < need || (need > 0 && !work)) return fail(TT_ENOSPC, "workspace %zu < %zu", work_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)work;
  double* Lb[2] = {(double*)base, (double*)(base + align_up(rp.left_max * 8))};
  double* Rb[2] = {(double*)(base + 2 * align_up(rp.left_max * 8)),
                   (double*)(base + 2 * align_up(rp.left_max * 8) + align_up(rp.right_max * 8))};
  const int h = rp.h;
  // L_1 = G_1 (I_1 x r_1); L_k = L_{k-1} (P_{k-1} x r_{k-1}) G_k (r_{k-1} x I_k r_k)
  const double* L = cores[0];
  for (int k = 2; k <= h; ++k) {
    double* dst = Lb[k & 1];
    HIP_OK(launch_gemm_smallk(L, cores[k - 1], dst, 0, prod(dims, 0, k - 1), dims[k - 1] * ranks[k],
                              (int)ranks[k - 1], st));
    L = dst;
  }
  // R_d = G_d (r_{d-1} x I_d); R_k = G_k (r_{k-1} I_k x r_k) R_{k+1} (r_k x Q_{k+1})
  const double* R = cores[d - 1];
  for (int k = d - 1; k >= h + 1; --k) {
    double* dst = Rb[k & 1];
    HIP_OK(launch_gemm_smallk(cores[k - 1], R, dst, 0, ranks[k - 1] * dims[k - 1], prod(dims, k, d),
                              (int)ranks[k], st));
    R = dst;
  }
  HIP_OK(launch_gemm_smallk(L, R, out, dtype == TT_F32, prod(dims, 0, h), prod(dims, h, d),
                            (int)ranks[h], st));
  return TT_OK;
}

}  // extern "C"

namespace {

// Backward of the reconstruction.  With the train split after core h, A =
// L_h R_{h+1} (L_h: P_h x r_h, the product of cores 1..h; R_{h+1}: r_h x
// Q_{h+1}, the product of cores h+1..d), and for L = <gout, A>:
//   dL_h = gout R_{h+1}^T  and  dR_{h+1} = L_h^T gout     (the two passes over gout)
// then the chain rule back through the partial products, recomputed from the
// cores (not kept from a forward call):
//   L_k = L_{k-1} G_k (P_{k-1} x I_k r_k):  dG_k = L_{k-1}^T dL_k,  dL_{k-1} = dL_k G_k^T
//   R_k = G_k R_{k+1} (r_{k-1} I_k x Q_{k+1}):  dG_k = dR_k R_{k+1}^T,  dR_{k+1} = G_k^T dR_k
// (dL_k and dR_k read in the reshaped shapes shown).  h is the first split
// with P_h >= Q_{h+1}, so that gout is a tall matrix for the two passes.
struct RecBwdPlan {
  int h;
  int64_t P[TT_MAX_D + 1];   // P[k] = I_1 ... I_k
  int64_t Q[TT_MAX_D + 2];   // Q[k] = I_k ... I_d (1-based), Q[d+1] = 1
  size_t off_L[TT_MAX_D + 1], off_R[TT_MAX_D + 1];
  size_t off_dL[2], off_dR[2], off_tmp, off_part;
  int64_t part_len;
  size_t bytes;
};

int recbwd_plan(int d, const int64_t* dims, const int64_t* ranks, RecBwdPlan& bp) {
  if (d < 2 || d > TT_MAX_D || !dims || !ranks) return fail(TT_EINVAL, "bad train description");
  if (ranks[0] != 1 || ranks[d] != 1) return fail(TT_EINVAL, "r_0 and r_d must be 1");
  for (int k = 0; k < d; ++k)
    if (dims[k] < 1) return fail(TT_EINVAL, "dims[%d] < 1", k);
  for (int k = 0; k <= d; ++k)
    if (ranks[k] < 1 || ranks[k] > kCMax) return fail(TT_EUNSUPPORTED, "rank %lld outside [1, 64]", (long long)ranks[k]);
  bp.P[0] = 1;
  for (int k = 1; k <= d; ++k) bp.P[k] = bp.P[k - 1] * dims[k - 1];
  bp.Q[d + 1] = 1;
  for (int k = d; k >= 1; --k) bp.Q[k] = bp.Q[k + 1] * dims[k - 1];
  bp.h = d - 1;
  for (int h = 1; h < d; ++h)
    if (bp.P[h] >= bp.Q[h + 1]) { bp.h = h; break; }
  const int h = bp.h;
  size_t off = 0;
  auto take = [&](int64_t doubles) { const size_t o = off; off += align_up((size_t)doubles * 8); return o; };
  for (int k = 2; k <= h; ++k) bp.off_L[k] = take(bp.P[k] * ranks[k]);           // L_k, k = 2..h
  for (int k = h + 1; k <= d - 1; ++k) bp.off_R[k] = take(ranks[k - 1] * bp.Q[k]);   // R_k, k = h+1..d-1
  int64_t maxL = 1, maxR = 1;
  for (int k = 1; k <= h; ++k) maxL = std::max(maxL, bp.P[k] * ranks[k]);
  for (int k = h + 1; k <= d; ++k) maxR = std::max(maxR, ranks[k - 1] * bp.Q[k]);
  bp.off_dL[0] = take(maxL);
  bp.off_dL[1] = take(maxL);
  bp.off_dR[0] = take(maxR);
  bp.off_dR[1] = take(maxR);
  const int64_t Qh = bp.Q[h + 1], rh = ranks[h];
  bp.off_tmp = take(Qh * rh);
  // partials: the second pass over gout, and every chain product
  const int nch = atb2_chunks(bp.P[h], (int)std::min<int64_t>(Qh, 1 << 30));
  int64_t part = nch > 1 ? (int64_t)nch * Qh * rh : 1;
  auto gpart = [&](int64_t M, int64_t N, int64_t K) {
    const int z = gemm_any_splits(M, N, K);
    if (z > 1) part = std::max(part, (int64_t)z * M * N);
  };
  for (int k = h; k >= 2; --k) {
    gpart(ranks[k - 1], dims[k - 1] * ranks[k], bp.P[k - 1]);
    gpart(bp.P[k - 1], ranks[k - 1], dims[k - 1] * ranks[k]);
  }
  for (int k = h + 1; k <= d - 1; ++k) {
    gpart(ranks[k - 1] * dims[k - 1], ranks[k], bp.Q[k + 1]);
    gpart(ranks[k], bp.Q[k + 1], ranks[k - 1] * dims[k - 1]);
  }
  bp.part_len = part;
  bp.off_part = take(part);
  bp.bytes = off;
  if (bp.P[h] > (int64_t)1 << 40 || Qh > (1 << 30)) return fail(TT_EUNSUPPORTED, "train too large");
  return TT_OK;
}

}  // namespace

extern "C" {

int tt_reconstruct_backward_workspace(int d, const int64_t* dims, const int64_t* ranks, size_t* bytes) {
  if (!bytes) return fail(TT_EINVAL, "bytes is NULL");
  RecBwdPlan bp;
  const int rc = recbwd_plan(d, dims, ranks, bp);
  if (rc) return rc;
  *bytes = bp.bytes;
  return TT_OK;
}

int tt_reconstruct_backward(int d, const int64_t* dims, const int64_t* ranks, const double* const* cores,
                            const void* gout, tt_dtype dtype, double* const* gcores, void* work, size_t work_bytes,
                            void* stream) {
  RecBwdPlan bp;
  int rc = recbwd_plan(d, dims, ranks, bp);
  if (rc) return rc;
  if (!cores || !gout || !gcores) return fail(TT_EINVAL, "cores/gout/gcores is NULL");
  if (dtype != TT_F64 && dtype != TT_F32) return fail(TT_EINVAL, "bad dtype");
  for (int k = 0; k < d; ++k)
    if (!cores[k] || !gcores[k]) return fail(TT_EINVAL, "cores[%d] or gcores[%d] is NULL", k, k);
  if (!work || work_bytes < bp.bytes) return fail(TT_ENOSPC, "workspace %zu < %zu", work_bytes, bp.bytes);
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)work;
  auto buf = [&](size_t off) { return (double*)(base + off); };
  const int h = bp.h;
  const int a_f32 = dtype == TT_F32;
  double* part = buf(bp.off_part);
  // left partial products L_2..L_h (L_1 = G_1) and right ones R_{d-1}..R_{h+1} (R_d = G_d)
  auto Lk = [&](int k) -> const double* { return k == 1 ? cores[0] : buf(bp.off_L[k]); };
  auto Rk = [&](int k) -> const double* { return k == d ? cores[d - 1] : buf(bp.off_R[k]); };
  for (int k = 2; k <= h; ++k)
    HIP_OK(launch_gemm_smallk(Lk(k - 1), cores[k - 1], buf(bp.off_L[k]), 0, bp.P[k - 1], dims[k - 1] * ranks[k],
                              (int)ranks[k - 1], st));
  for (int k = d - 1; k >= h + 1; --k)
    HIP_OK(launch_gemm_smallk(cores[k - 1], Rk(k + 1), buf(bp.off_R[k]), 0, ranks[k - 1] * dims[k - 1], bp.Q[k + 1],
                              (int)ranks[k], st));
  const int64_t Ph = bp.P[h], Qh = bp.Q[h + 1];
  const int rh = (int)ranks[h];
  // pass 1: dL_h = gout R_{h+1}^T (R_{h+1}, r_h x Q column-major, is the k-major right operand)
  double* dL = (h == 1) ? gcores[0] : buf(bp.off_dL[h & 1]);
  HIP_OK(launch_ax(gout, a_f32, Rk(h + 1), dL, 0, Ph, (int)Qh, rh, COL, ax_chunks(Ph, (int)Qh, rh), nullptr,
                   nullptr, nullptr, st));
  // pass 2: dR_{h+1}^T = gout^T L_h (Q x r_h), then transposed to r_h x Q
  {
    const int nch = atb2_chunks(Ph, (int)Qh);
    double* tmp = buf(bp.off_tmp);
    HIP_OK(launch_atb2(gout, a_f32, Lk(h), 0, Ph, (int)Qh, rh, COL, 0, nch == 1 ? tmp : part, nch, st));
    if (nch > 1) HIP_OK(launch_reduce(part, nch, Qh * rh, tmp, nullptr, st));
    double* dR = (h + 1 == d) ? gcores[d - 1] : buf(bp.off_dR[(h + 1) & 1]);
    HIP_OK(launch_transpose(tmp, Qh, rh, dR, st));
  }
  // back through the left products: dL_k read as dM (P_{k-1} x I_k r_k)
  for (int k = h; k >= 2; --k) {
    const double* dM = buf(bp.off_dL[k & 1]);
    const int64_t P = bp.P[k - 1], ra = ranks[k - 1], J = dims[k - 1] * ranks[k];
    // dG_k (r_{k-1} x I_k r_k) = L_{k-1}^T dM
    HIP_OK(launch_gemm_any(Lk(k - 1), P, 1, dM, 1, P, gcores[k - 1], ra, J, P, part, gemm_any_splits(ra, J, P), st));
    // dL_{k-1} (P_{k-1} x r_{k-1}) = dM G_k^T (G_k read as r_{k-1} x I_k r_k)
    double* dst = (k == 2) ? gcores[0] : buf(bp.off_dL[(k - 1) & 1]);
    HIP_OK(launch_gemm_any(dM, 1, P, cores[k - 1], ra, 1, dst, P, ra, J, part, gemm_any_splits(P, ra, J), st));
  }
  // back through the right products: dR_k read as dN (r_{k-1} I_k x Q_{k+1})
  for (int k = h + 1; k <= d - 1; ++k) {
    const double* dN = buf(bp.off_dR[k & 1]);
    const int64_t X = ranks[k - 1] * dims[k - 1], rb = ranks[k], Q = bp.Q[k + 1];
    // dG_k (r_{k-1} I_k x r_k) = dN R_{k+1}^T
    HIP_OK(launch_gemm_any(dN, 1, X, Rk(k + 1), rb, 1, gcores[k - 1], X, rb, Q, part, gemm_any_splits(X, rb, Q), st));
    // dR_{k+1} (r_k x Q_{k+1}) = G_k^T dN (G_k read as r_{k-1} I_k x r_k)
    double* dst = (k + 1 == d) ? gcores[d - 1] : buf(bp.off_dR[(k + 1) & 1]);
    HIP_OK(launch_gemm_any(cores[k - 1], X, 1, dN, 1, X, dst, rb, Q, X, part, gemm_any_splits(rb, Q, X), st));
  }
  return TT_OK;
}

static int train_checks(int d, const int64_t* dims, const int64_t* ranks, tt_dtype dtype) {
  if (d < 2 || d > TT_MAX_D || !dims || !ranks) return fail(TT_EINVAL, "bad train description");
  for (int k = 0; k < d; ++k)
    if (dims[k] < 1) return fail(TT_EINVAL, "dims[%d] < 1", k);
  for (int k = 0; k <= d; ++k)
    if (ranks[k] < 1 || ranks[k] > kCMax) return fail(TT_EUNSUPPORTED, "rank %lld outside [1, 64]", (long long)ranks[k]);
  if (ranks[0] != 1 || ranks[d] != 1) return fail(TT_EINVAL, "r_0 and r_d must be 1");
  if (dtype != TT_F64 && dtype != TT_F32) return fail(TT_EINVAL, "bad core dtype");
  // the one-sample-per-thread kernels hold vectors of up to 32 entries; wider
  // trains take the wave-per-sample kernels, which read FP64 cores only
  if (dtype == TT_F32 && sample_rm(d, ranks) == 0)
    return fail(TT_EUNSUPPORTED, "FP32 cores need every rank <= 32");
  return TT_OK;
}

int tt_sample(int d, const int64_t* dims, const int64_t* ranks, const void* const* cores, tt_dtype core_dtype,
              const int64_t* idx, int64_t N, double* out, void* stream) {
  int rc = train_checks(d, dims, ranks, core_dtype);
  if (rc) return rc;
  if (!cores) return fail(TT_EINVAL, "cores is NULL");
  if (N < 0) return fail(TT_EINVAL, "N < 0");
  if (N > 0 && (!idx || !out)) return fail(TT_EINVAL, "idx/out is NULL");
  for (int k = 0; k < d; ++k)
    if (!cores[k]) return fail(TT_EINVAL, "cores[%d] is NULL", k);
  if (sample_rm(d, ranks))
    HIP_OK(launch_sample2(d, dims, ranks, cores, core_dtype == TT_F32, idx, N, out, (hipStream_t)stream));
  else
    HIP_OK(launch_sample(d, dims, ranks, (const double* const*)cores, idx, N, out, (hipStream_t)stream));
  return TT_OK;
}

int tt_sample_backward_workspace(int d, const int64_t* dims, const int64_t* ranks, int64_t N, size_t* bytes) {
  if (!bytes) return fail(TT_EINVAL, "bytes is NULL");
  int rc = train_checks(d, dims, ranks, TT_F64);
  if (rc) return rc;
  if (N < 0) return fail(TT_EINVAL, "N < 0");
  *bytes = sample_rm(d, ranks) ? sample_bwd2_workspace(d, dims, ranks, N) : 0;
  return TT_OK;
}

static int sample_bwd(int d, const int64_t* dims, const int64_t* ranks, const void* const* left,
                      const void* const* right, tt_dtype dtype, const int64_t* idx, int64_t N, const double* gout,
                      void* const* gcores, void* work, size_t work_bytes, void* stream) {
  int rc = train_checks(d, dims, ranks, dtype);
  if (rc) return rc;
  if (!left || !right || !gcores) return fail(TT_EINVAL, "cores/gcores is NULL");
  for (int k = 0; k < d; ++k)
    if (!left[k] || !right[k] || !gcores[k]) return fail(TT_EINVAL, "core or gradient pointer %d is NULL", k);
  if (N < 0) return fail(TT_EINVAL, "N < 0");
  if (N > 0 && (!idx || !gout)) return fail(TT_EINVAL, "idx/gout is NULL");
  hipStream_t st = (hipStream_t)stream;
  if (sample_rm(d, ranks)) {
    const size_t need = sample_bwd2_workspace(d, dims, ranks, N);
    if (!work || work_bytes < need) return fail(TT_ENOSPC, "workspace %zu bytes < %zu needed", work_bytes, need);
    HIP_OK(launch_sample_bwd2(d, dims, ranks, left, right, dtype == TT_F32, idx, N, gout, gcores, work, work_bytes,
                              st));
  } else {
    HIP_OK(launch_sample_bwd(d, dims, ranks, (const double* const*)left,
                             right == left ? nullptr : (const double* const*)right, idx, N, gout,
                             (double* const*)gcores, st));
  }
  return TT_OK;
}

int tt_sample_backward(int d, const int64_t* dims, const int64_t* ranks, const void* const* cores,
                       tt_dtype core_dtype, const int64_t* idx, int64_t N, const double* gout, void* const* gcores,
                       void* work, size_t work_bytes, void* stream) {
  return sample_bwd(d, dims, ranks, cores, cores, core_dtype, idx, N, gout, gcores, work, work_bytes, stream);
}

int tt_sample_backward_mixed(int d, const int64_t* dims, const int64_t* ranks, const void* const* left_cores,
                             const void* const* right_cores, tt_dtype core_dtype, const int64_t* idx, int64_t N,
                             const double* gout, void* const* gcores, void* work, size_t work_bytes, void* stream) {
  if (!right_cores) return fail(TT_EINVAL, "right_cores is NULL");
  return sample_bwd(d, dims, ranks, left_cores, right_cores, core_dtype, idx, N, gout, gcores, work, work_bytes,
                    stream);
}

// ---- completion steps (Sec. 4.3) -------------------------------------------
static_assert(TT_REDUCE_WORK_BYTES >= 2 * 256 * sizeof(double), "partials of the reductions");

static int reduce_checks(int64_t N, const void* work, size_t work_bytes) {
  if (N < 0) return fail(TT_EINVAL, "N < 0");
  if (!work || work_bytes < TT_REDUCE_WORK_BYTES || work_bytes < reduce_workspace_bytes())
    return fail(TT_ENOSPC, "work %zu bytes < %d needed", work_bytes, TT_REDUCE_WORK_BYTES);
  return TT_OK;
}

int tt_residual(int64_t N, const double* pred, const double* vals, double* z, double* f, void* work,
                size_t work_bytes, void* stream) {
  int rc = reduce_checks(N, work, work_bytes);
  if (rc) return rc;
  if (!f) return fail(TT_EINVAL, "f is NULL");
  if (N > 0 && (!pred || !vals || !z)) return fail(TT_EINVAL, "pred/vals/z is NULL");
  HIP_OK(launch_residual(pred, vals, N, z, f, (double*)work, (hipStream_t)stream));
  return TT_OK;
}

int tt_line_step(int64_t N, const double* p, const double* z, double* out, void* work, size_t work_bytes,
                 void* stream) {
  int rc = reduce_checks(N, work, work_bytes);
  if (rc) return rc;
  if (!out) return fail(TT_EINVAL, "out is NULL");
  if (N > 0 && (!p || !z)) return fail(TT_EINVAL, "p/z is NULL");
  HIP_OK(launch_line_step(p, z, N, out, (double*)work, (hipStream_t)stream));
  return TT_OK;
}

int tt_axpy(int64_t n, double a, const double* a_dev, const double* x, double* y, void* stream) {
  if (n < 0) return fail(TT_EINVAL, "n < 0");
  if (n > 0 && (!x || !y)) return fail(TT_EINVAL, "x/y is NULL");
  HIP_OK(launch_axpy(n, a, a_dev, x, y, (hipStream_t)stream));
  return TT_OK;
}

static int manifold_checks(int d, const int64_t* dims, const int64_t* ranks, const double* const* a,
                           const double* const* b, const double* const* c, double* const* out) {
  int rc = train_checks(d, dims, ranks, TT_F64);
  if (rc) return rc;
  if (!a || !b || !out) return fail(TT_EINVAL, "a core list is NULL");
  for (int k = 0; k < d; ++k)
    if (!a[k] || !b[k] || !out[k] || (c && !c[k])) return fail(TT_EINVAL, "core pointer %d is NULL", k);
  return TT_OK;
}

int tt_tangent_project(int d, const int64_t* dims, const int64_t* ranks, const double* const* U,
                       const double* const* G, double* const* dC, void* stream) {
  int rc = manifold_checks(d, dims, ranks, U, G, nullptr, dC);
  if (rc) return rc;
  HIP_OK(launch_tangent_project(d, dims, ranks, U, G, dC, (hipStream_t)stream));
  return TT_OK;
}

int tt_tangent_train(int d, const int64_t* dims, const int64_t* ranks, const double* const* U,
                     const double* const* V, const double* const* dC, double t_host, const double* t_dev,
                     int with_base, double* const* W, void* stream) {
  if (!dC) return fail(TT_EINVAL, "dC is NULL");
  int rc = manifold_checks(d, dims, ranks, U, V, dC, W);
  if (rc) return rc;
  HIP_OK(launch_tangent_train(d, dims, ranks, U, V, dC, t_host, t_dev, with_base ? 1 : 0, W,
                              (hipStream_t)stream));
  return TT_OK;
}

}  // extern "C"
