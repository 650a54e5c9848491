/*
 * ttutv.h -- C ABI of the TT-UTV library for AMD Instinct MI355X (gfx950).
 *
 * TT-UTV (Wang, Che & Wei, "Effective algorithms for tensor-train
 * decomposition via the UTV framework") computes a tensor train by a sweep of
 * truncated rank-revealing UTV factorisations of the unfoldings, in place of
 * the SVDs of TT-SVD.  The inner factorisation here is a randomized
 * power-iteration UTV: a Gaussian test matrix on the core side of the
 * unfolding, q power steps, a Rayleigh-Ritz step on the ell-dimensional
 * subspace it spans, and truncation at a fixed rank or at the rank rule that
 * follows Alg. 2.
 *
 * Conventions shared by every entry point
 *  - Tensors are flat in reverse lexicographic order (the paper's `ivec`:
 *    i1 fastest, Sec. 2.1).  A C-contiguous array of shape (I_d, ..., I_1) has
 *    this layout.
 *  - TT core k (1-based) has shape r_{k-1} x I_k x r_k and is stored
 *    column-major: element (a, i, b) at a + r_{k-1} * (i + I_k * b)
 *    (the core of Eq. (TT), reshaped as MATLAB's reshape does).
 *  - ranks arrays hold r_0..r_d (d+1 entries, r_0 = r_d = 1).
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer.  The
 *    library never allocates or frees device memory; it enqueues work on the
 *    given HIP stream (NULL = default stream).
 *  - Every function returns TT_OK (0) or a negative status; on error
 *    tt_last_error() returns a message (thread-local, valid until the next
 *    call from the same thread).  Argument errors are detected on the host
 *    before any work is enqueued.
 */
#ifndef TTUTV_H
#define TTUTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_OK 0
#define TT_EINVAL (-1)        /* bad argument: dims, ranks, enum value, null pointer */
#define TT_ENOSPC (-2)        /* workspace smaller than tt_utv_workspace reported */
#define TT_ERANK (-3)         /* eps not reachable within max_rank; cores and report still written */
#define TT_ENONFINITE (-4)    /* input holds NaN or Inf (detected from ||A||_F after the
                                 first pass over A; the sweep stops there) */
#define TT_EHIP (-5)          /* a HIP runtime call failed */
#define TT_EUNSUPPORTED (-6)  /* valid request outside the library's limits (e.g. ell > 64) */

#define TT_MAX_D 32           /* largest tensor order */
#define TT_MAX_ELL 64         /* largest sketch width ell (and therefore rank) */

typedef enum { TT_L2R = 0, TT_R2L = 1 } tt_sweep;
/* TT_ULV + TT_L2R: Alg. 1 (fixed ranks) / Alg. 2 (prescribed accuracy).
 * TT_URV + TT_R2L: Alg. 3 and its prescribed-accuracy form (Sec. 3.2).
 * TT_URV + TT_L2R: the index-reversal form (remark after Thm. 3.2).
 * TT_ULV + TT_R2L: Alg. 4 (appendix), carry U^ L11 without the U2 L21 term.
 * TT_SVD: truncated SVD of every unfolding (TT-SVD): the exact ell = n case
 * where the core side n is at most 64; wider core sides take subspace
 * iteration on the leading 64 directions (30 power steps, then Rayleigh-Ritz:
 * the leading singular subspace to rounding when s_65 <= 0.54 s_r), ranks up
 * to 64. */
typedef enum { TT_ULV = 0, TT_URV = 1, TT_SVD = 2 } tt_variant;
typedef enum { TT_F64 = 0, TT_F32 = 1 } tt_dtype;

typedef struct {
  int32_t q;                /* power steps (>= 0) */
  int32_t oversample;       /* p: ell = min(r + p, n, m) */
  uint64_t seed;            /* seed of the Gaussian test matrices */
  int32_t max_rank;         /* eps mode: rank cap per step (0 = TT_MAX_ELL) */
  int32_t exact_delta;      /* 1: measure every step error ||C - C_r||_F by an extra
                               pass over C; 0: from ||C||^2 - ||carry||^2, an estimate
                               that loses digits by cancellation when a step error is
                               below ~1e-7 ||C|| (err_bound is then an estimate too;
                               with 1 it is a bound) */
  const double* weights;    /* host, d-1 entries with sum w_k^2 = 1, or NULL for the
                               default (1/sqrt(d-1); 1/(d-1) for Alg. 4) */
  int32_t profile;          /* bit mask of kernel classes (bit c = class c,
                               TT_PROFILE_ALL = every class) whose launches are timed
                               with HIP events on the caller's stream, filling
                               tt_report.kstat; 0 = no events */
  int32_t prec;             /* tt_prec: TT_PREC_FP64, TT_PREC_MIXED or TT_PREC_MIXED_BF16 */
  int32_t fuse_ata;         /* 1: a power step over FP64 data stored column-major
                               (right-to-left sweeps) with n <= 512, ell <= 32 and
                               n ell <= 12288 forms A^T (A X) with one read of A
                               (class "tall_ata"); 0 (default): two passes, A X then
                               A^T Y, which measure faster at n = 512: the one-pass
                               kernel can hold only 16-row tiles of A on chip, and
                               128-byte column segments stream at about 2 TB/s */
  int32_t orth;             /* tt_orth: orthonormaliser of the intermediate power
                               iterates (the last one before the Rayleigh-Ritz step
                               always takes Householder QR) */
  int32_t separate_sketch;  /* 0 (default): in the right-to-left sweep, when a step
                               in Gram mode (n <= 64) is followed by a sketched step,
                               the carry pass also forms the next step's first
                               sketch product Y = A_next G (A_next = the carry,
                               reshaped) from the same reading of the unfolding,
                               through Y = sum_i A_i (V1 G_i) over the row slabs A_i;
                               the next step then starts from Y instead of reading
                               the carry once more (carry rank <= 32, sketch width
                               <= 48, n <= 48 in the FP64 form / 64 in the mixed
                               form; otherwise, or with the BF16 or one-pass power
                               products, the passes stay separate).  1: always a
                               separate sketch pass. */
  int32_t inner;            /* tt_inner: the truncated factorisation of each step */
} tt_opts;

/* TT_INNER_SKETCH: the randomized power-iteration factorisation (a Gaussian
 * test matrix of ell = r + p columns, q power steps, Rayleigh-Ritz).
 * TT_INNER_DEFLATION: one core-side vector at a time, the paper's USV-plus
 * based TT-ULV (Sec. 3.3 cost model 4 m n (k+1) q; Sec. 4): on the tall
 * orientation A (m x n) of the unfolding, vector j starts from column j of the
 * same Gaussian test matrix with the vectors already found projected out (two
 * rounds of classical Gram-Schmidt), takes q >= 1 power steps
 * x <- P(A^T A x) / ||P(A^T A x)||, and adds ||A v_j||^2 to the kept energy;
 * the search stops at the fixed rank, or at the first j with
 * ||C||^2 - kept <= eps_k^2 (the rank rule after Alg. 2), or after
 * min(n, m, max_rank or TT_MAX_ELL) vectors.  The vectors are orthonormal, so
 * delta_k^2 = ||C||^2 - ||carry||^2 as with the sketch.  Steps with n <= 64
 * form A^T A in one pass and search on it in one workgroup; wider steps read A
 * once per power step (class "defl_pass", n <= 4096; with a prescribed
 * accuracy the check applies to the largest n a step can reach, the rank cap
 * times I_k, so wide modes need max_rank, else TT_EUNSUPPORTED).  FP64 form only; not
 * with Alg. 4 (TT_ULV + TT_R2L) or TT_SVD (TT_EINVAL); report.ell holds the
 * number of vectors kept and report.sweeps 0. */
typedef enum { TT_INNER_SKETCH = 0, TT_INNER_DEFLATION = 1 } tt_inner;

/* TT_ORTH_HOUSEHOLDER: Householder QR (one workgroup, or a tree of block QRs
 * for iterates taller than one workgroup holds).
 * TT_ORTH_CHOLQR: shifted CholeskyQR (after Fukaya et al., SIAM J. Sci.
 * Comput. 2020), three rounds of Gram matrix M^T M (FP64, streaming kernel),
 * Cholesky factor R of M^T M + s I and its inverse in one wave, M <- M R^{-1},
 * with s = 11 (n ell + ell (ell + 1)) 2^-53 tr(M^T M): positive definite for
 * iterates conditioned up to about 2^53 (power iterates of noisy tensors
 * reach 1e14), each round squaring down the condition number, and finite for
 * exactly rank-deficient iterates.  The result spans the same space as M and
 * is orthonormal to about the shift's size; only the basis differs from
 * Householder's, and the Rayleigh-Ritz step after the last (Householder)
 * iterate does not depend on it. */
typedef enum { TT_ORTH_HOUSEHOLDER = 0, TT_ORTH_CHOLQR = 1 } tt_orth;

/* TT_PREC_FP64: every carry, sketch and product in FP64.
 * TT_PREC_MIXED: carries and power iterates stored in FP32 (half the traffic
 * of every pass after the first); the power products run on FP32 matrix cores
 * (FP32 operands and accumulation); the final Rayleigh-Ritz pass reads A with
 * FP64 accumulation, and its Gram matrix, the factorisations and the rank rule
 * stay FP64.  Steps whose core side n is at most 64 form A^T A in one FP64
 * pass (it decides the rank and must be accurate to eps^2) and run no
 * low-precision product: there the mixed form differs from TT_PREC_FP64 only
 * in the FP32 storage of the carry.  Storing carry k in FP32 perturbs it by
 * rho_k <= 2^-24 ||carry_k|| (measured exactly); the report's err_bound is then
 * sqrt(sum delta_k^2) + sum rho_k (sum delta_k + sum rho_k for Alg. 4).  With
 * a prescribed accuracy the rank rule aims at eps - (d-2) 2^-24 (the a-priori
 * budget of the d-2 FP32 carries), so err_bound <= eps ||A||_F still holds;
 * eps at or below that budget is rejected (TT_EINVAL), and with measured step
 * errors (exact_delta = 1) a bound above eps ||A||_F clears rank_rule_met and
 * returns TT_ERANK (without them the bound is an estimate and is not checked).
 * TT_PREC_MIXED_BF16: as TT_PREC_MIXED with the power products on BF16
 * operands (FP32 accumulation): the sketch resolves singular directions only
 * to about 4e-3 of the largest, which costs rank (or, under a rank cap, the
 * tolerance) at prescribed accuracies below about 1e-3; the bound stays valid. */
typedef enum { TT_PREC_FP64 = 0, TT_PREC_MIXED = 1, TT_PREC_MIXED_BF16 = 2 } tt_prec;

/* Kernel classes of the profile (tt_kernel_class_name gives their names). */
#define TT_NKCLASS 9
#define TT_PROFILE_ALL ((1 << TT_NKCLASS) - 1)
typedef struct {
  int64_t launches;
  double ms;        /* summed launch durations (HIP events around each launch) */
  double bytes;     /* algorithmic bytes: operands read once + results written */
  double flops;     /* algorithmic floating-point operations */
} tt_kstat;

typedef struct {
  int64_t ranks[TT_MAX_D + 1];  /* r_0..r_d actually used */
  int64_t ell[TT_MAX_D];        /* sketch width of unfolding k (index k-1) */
  double delta[TT_MAX_D];       /* step error of unfolding k: ||C - truncated||_F */
  double normC[TT_MAX_D];       /* ||C||_F of the matrix factorised for unfolding k */
  double norm_A;                /* ||A||_F */
  double err_bound;             /* sqrt(sum delta^2) (Cor. 3.1 / Thm. 3.2), or
                                   sum delta for Alg. 4 (Prop. A.1) */
  int32_t rank_rule_met;        /* eps mode: 1 if every step met its tolerance */
  int32_t d;
  tt_kstat kstat[TT_NKCLASS];   /* classes selected by opts.profile */
  int32_t sweeps[TT_MAX_D];     /* Jacobi sweeps of the Rayleigh-Ritz step of unfolding k */
  double rho[TT_MAX_D];         /* mixed forms: ||carry - fl32(carry)||_F of unfolding k */
  int32_t err_bound_measured;   /* 1: every delta was measured directly (opts.exact_delta)
                                   and err_bound is a bound; 0: the deltas are the estimates
                                   sqrt(||C||^2 - ||carry||^2), and so is err_bound */
} tt_report;

/* Name of kernel class c (0 <= c < TT_NKCLASS), or NULL. */
const char* tt_kernel_class_name(int c);

/* Fills opts with q = 1, oversample = 8, seed = 0, max_rank = 0,
 * exact_delta = 0, weights = NULL, profile = 0, prec = TT_PREC_FP64,
 * fuse_ata = 0, orth = TT_ORTH_HOUSEHOLDER, separate_sketch = 0,
 * inner = TT_INNER_SKETCH. */
void tt_default_opts(tt_opts* opts);

/* Device bytes of workspace tt_utv_decompose needs for this problem.
 * ranks (host, d+1) for fixed ranks, or NULL with eps >= 0 for prescribed
 * accuracy (then the bound assumes every rank reaches its cap). */
int tt_utv_workspace(int d, const int64_t* dims, const int64_t* ranks, double eps,
                     tt_sweep sweep, tt_variant variant, tt_dtype dtype,
                     const tt_opts* opts, size_t* bytes);

/* Largest number of doubles core k (0-based) can need: max r_{k-1} * I_k * r_k
 * over the ranks this problem may produce (exact for fixed ranks). */
int tt_utv_core_capacity(int d, const int64_t* dims, const int64_t* ranks, double eps,
                         const tt_opts* opts, int64_t* capacity /* host, d entries */);

/* TT-UTV decomposition (Alg. 1-4 and the prescribed-accuracy forms).
 *  A          device, prod(dims) elements of `dtype`, ivec order; not modified.
 *  dims       host, d extents (each >= 1), 2 <= d <= TT_MAX_D.
 *  ranks      host, r_0..r_d for fixed ranks (clamped to what each unfolding
 *             allows, as the theorems allow ranks "not higher than" r_k), or
 *             NULL for prescribed accuracy eps (relative: ||A - A_TT||_F <=
 *             eps ||A||_F, eps_k = w_k eps ||A||_F per step).
 *  work       device workspace of at least tt_utv_workspace bytes.
 *  cores      host array of d device pointers; core k receives r_{k-1} I_k r_k
 *             doubles (see tt_utv_core_capacity), layout above.
 *  rep        host, filled on TT_OK and TT_ERANK (may be NULL).
 *  stream     hipStream_t or NULL.
 * With fixed ranks the call synchronises the stream twice: after the first
 * pass over A (a non-finite input stops the sweep there with TT_ENONFINITE)
 * and at the end, to fill the report; with eps it also synchronises after
 * every step to size the next one (and, with the deflation inner kernel,
 * after every vector of a streaming step).  With fixed ranks, rep == NULL and
 * opts.profile = 0 it only enqueues kernels on the stream and never waits on
 * it, so the call can be recorded into a HIP graph; a non-finite input is
 * then not reported and leaves non-finite cores. */
int tt_utv_decompose(const void* A, tt_dtype dtype, int d, const int64_t* dims,
                     const int64_t* ranks, double eps, tt_sweep sweep, tt_variant variant,
                     const tt_opts* opts, void* work, size_t work_bytes,
                     double* const* cores, tt_report* rep, void* stream);

/* Bytes of the static device scratch of tt_utv_decompose_noalloc. */
#define TT_NOALLOC_SCRATCH_BYTES (64u << 20)

/* tt_utv_decompose without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a static device array
 * of TT_NOALLOC_SCRATCH_BYTES (64 MiB) that every device the library runs on
 * holds until the process ends; a problem whose tt_utv_workspace exceeds it
 * returns TT_ENOSPC before any work is enqueued.  opts.profile must be 0 (it
 * would create HIP events).  Otherwise arguments, results, report and
 * synchronisation are those of tt_utv_decompose, whose kernels it runs (so
 * only a fixed-rank call with rep == NULL can be recorded into a graph, after
 * a first call on the device has looked up the scratch);
 * nothing in the scratch needs to start cleared.  All calls on one device
 * share its scratch: calls that overlap in time on one device (other host
 * threads, or other streams before this call's work has finished) race and
 * give undefined results.  Calls no hipMalloc/hipFree or other allocating
 * routine; the first call on each device looks up the scratch's address. */
int tt_utv_decompose_noalloc(const void* A, tt_dtype dtype, int d, const int64_t* dims,
                             const int64_t* ranks, double eps, tt_sweep sweep, tt_variant variant,
                             const tt_opts* opts, double* const* cores, tt_report* rep, void* stream);

/* Device bytes of workspace tt_reconstruct needs for this train. */
int tt_reconstruct_workspace(int d, const int64_t* dims, const int64_t* ranks, size_t* bytes);

/* Full tensor from TT cores, Eq. (TT).  cores: host array of d device
 * pointers (FP64, layout above); ranks r_0..r_d with every r_k <= 64; out:
 * device, prod(dims) elements of `dtype` in ivec order; work: device
 * workspace of tt_reconstruct_workspace bytes (the two partial products of
 * the train, split near the middle so that out = L R is one GEMM).
 * Enqueues only. */
int tt_reconstruct(int d, const int64_t* dims, const int64_t* ranks,
                   const double* const* cores, void* out, tt_dtype dtype,
                   void* work, size_t work_bytes, void* stream);

/* Device bytes of workspace tt_reconstruct_backward needs for this train. */
int tt_reconstruct_backward_workspace(int d, const int64_t* dims, const int64_t* ranks, size_t* bytes);

/* Gradient of L = <gout, A_TT> with respect to every core, A_TT the dense
 * tensor of Eq. (TT) (Sec. 2.1): dL/dG_k(a, i, b) = sum over the modes before
 * and after k of Left_k(p, a) gout(p, i, q) Right_k(b, q), Left_k and Right_k
 * the products of the cores before and after k.  gout: device, prod(dims)
 * elements of `dtype` in ivec order (the upstream gradient of tt_reconstruct);
 * gcores[k]: device, r_{k-1} I_k r_k doubles, overwritten with dL/dG_k in the
 * core layout above; cores: FP64, every r_k <= 64.  The partial products of
 * the train are recomputed from the cores (nothing is kept from a forward
 * call): gout is read twice (gout Right^T and Left^T gout at one split of the
 * train), then the chain rule runs back through the smaller partial products.
 * Sums run in a fixed order (bitwise reproducible).  work: device workspace of
 * tt_reconstruct_backward_workspace bytes.  Enqueues only. */
int tt_reconstruct_backward(int d, const int64_t* dims, const int64_t* ranks, const double* const* cores,
                            const void* gout, tt_dtype dtype, double* const* gcores, void* work,
                            size_t work_bytes, void* stream);

/* Entries of the train at N multi-indices, Eq. (TT).  cores: host array of d
 * device pointers of `core_dtype` (TT_F64 or TT_F32; layout above); idx:
 * device, N x d int64 row-major, 0-based, each i_k < I_k (not checked on the
 * device: the caller guarantees it); out: device, N doubles (FP64 products).
 * With every rank <= 32 each thread carries one sample's running row vector
 * in registers, the cores staged once per workgroup in LDS when they fit;
 * wider trains (ranks up to 64, FP64 cores only) take one wave per sample.
 * Enqueues only. */
int tt_sample(int d, const int64_t* dims, const int64_t* ranks, const void* const* cores,
              tt_dtype core_dtype, const int64_t* idx, int64_t N, double* out, void* stream);

/* Device bytes of workspace tt_sample_backward(_mixed) needs for N samples of
 * this train (0 when a rank exceeds 32). */
int tt_sample_backward_workspace(int d, const int64_t* dims, const int64_t* ranks, int64_t N,
                                 size_t* bytes);

/* Gradient of L = sum_s gout[s] * A_TT[idx_s] with respect to every core, the
 * derivative of Eq. (TT) at the sampled entries: dL/dG_k(a, i, b) = sum over
 * the samples with i_k = i of gout[s] Left_k^s(a) Right_k^s(b), Left_k^s =
 * G_1[i_1] ... G_{k-1}[i_{k-1}] and Right_k^s = G_{k+1}[i_{k+1}] ... G_d[i_d].
 * gcores[k] (device, same type, layout and size as core k) is overwritten.
 * The interface products of each sample are recomputed from the cores (not
 * kept from a forward call) into `work` (tt_sample_backward_workspace bytes,
 * in blocks of at most 2^20 samples); each of 256 workgroups takes a
 * contiguous share of the samples, every 16 x 16 tile of a gradient slice is
 * owned by one wave, which feeds it the samples of that slice in sample order,
 * four per FP64 matrix-core step, and the workgroups' partials are summed in a
 * fixed order: the result is bitwise reproducible.  Trains with a rank above
 * 32 use FP64 atomics instead (not reproducible bitwise; work unused).
 * Enqueues only. */
int tt_sample_backward(int d, const int64_t* dims, const int64_t* ranks,
                       const void* const* cores, tt_dtype core_dtype, const int64_t* idx, int64_t N,
                       const double* gout, void* const* gcores, void* work, size_t work_bytes,
                       void* stream);

/* The same gradient taken at the mixed-canonical points of one train, the
 * ingredient of its Riemannian gradient (Sec. 4.3, RGrad for completion):
 * gcores[k] = dL/dC_k of L = sum_s gout[s] * (L_1..L_{k-1} C_k R_{k+1}..R_d)[idx_s],
 * where L_j = left_cores[j] (left-orthogonal form) and R_j = right_cores[j]
 * (right-orthogonal form of the same train, same ranks); with left_cores ==
 * right_cores it is tt_sample_backward.  Same layouts, checks, workspace and
 * stream behaviour as tt_sample_backward. */
int tt_sample_backward_mixed(int d, const int64_t* dims, const int64_t* ranks,
                             const void* const* left_cores, const void* const* right_cores,
                             tt_dtype core_dtype, const int64_t* idx, int64_t N, const double* gout,
                             void* const* gcores, void* work, size_t work_bytes, void* stream);

const char* tt_last_error(void);

/* ---- Completion steps on TT cores (Sec. 4.3, "MRI data completion") ------
 * Vectors are device arrays of FP64; `work` is caller-owned device memory of
 * at least TT_REDUCE_WORK_BYTES bytes (partial sums); every sum is a sum of
 * per-workgroup partials in a fixed order (bitwise reproducible); each call
 * only enqueues work on `stream` and results stay on the device.
 * Errors: TT_EINVAL (N < 0, a NULL pointer where data is needed, a bad train
 * description), TT_ENOSPC (work smaller than TT_REDUCE_WORK_BYTES),
 * TT_EUNSUPPORTED (a rank above 64). */
#define TT_REDUCE_WORK_BYTES 4096

/* z = pred - vals over N sampled entries and f[0] = sum_s z_s^2 / 2: the
 * residual and objective of the completion problem f = 1/2 ||P_Omega(X - M)||^2.
 * z may alias pred. */
int tt_residual(int64_t N, const double* pred, const double* vals, double* z, double* f, void* work,
                size_t work_bytes, void* stream);

/* out[0] = alpha = <p, z> / <p, p> (0 when p = 0), out[1] = <p, z>,
 * out[2] = <p, p>: the exact minimiser of 1/2 ||z - alpha p||^2, i.e. of f on
 * the line X - alpha xi whose sampled direction is p = P_Omega(xi) (the step
 * size of the Riemannian gradient iteration, and of gradient descent on the
 * cores with p the sampled directional derivative). */
int tt_line_step(int64_t N, const double* p, const double* z, double* out, void* work, size_t work_bytes,
                 void* stream);

/* y += a * s * x over n entries, with s = *a_dev when a_dev is not NULL (a
 * scalar computed on the device, such as out[0] of tt_line_step) and s = 1
 * otherwise. */
int tt_axpy(int64_t n, double a, const double* a_dev, const double* x, double* y, void* stream);

/* Projection onto the tangent space of the manifold of trains of fixed ranks
 * at X = U_1 ... U_d, where U_1 .. U_{d-1} are left-orthogonal (Def. 2.2), of
 * the core gradients G_k taken at the mixed-canonical points of X
 * (tt_sample_backward_mixed with the left- and right-orthogonal forms): on
 * the left unfoldings ((r_{k-1} I_k) x r_k), dC_k = (I - U_k U_k^T) G_k for
 * k < d, and dC_d = G_d.  All cores FP64, column-major (r_{k-1}, I_k, r_k),
 * device; dC[k] may not alias G[k] or U[k].  Ranks <= 64. */
int tt_tangent_project(int d, const int64_t* dims, const int64_t* ranks, const double* const* U,
                       const double* const* G, double* const* dC, void* stream);

/* Cores of t xi (with_base = 0) or of X + t xi (with_base = 1), where
 * xi = sum_k U_1..U_{k-1} dC_k V_{k+1}..V_d is the tangent vector of
 * tt_tangent_project and V the right-orthogonal form of X: ranks
 * (1, 2 r_1, ..., 2 r_{d-1}, 1), first core [t dC_1, U_1], interior cores
 * [[V_k, 0], [t dC_k, U_k]], last core [[V_d], [t dC_d (+ U_d)]] (blocks
 * stacked along the rank indices).  t = t_host * (*t_dev) when t_dev is not
 * NULL, else t_host.  W[k] (device, FP64, column-major) holds
 * w_{k-1} I_k w_k doubles with w = (1, 2 r_1, ..., 2 r_{d-1}, 1).  Ranks <= 64
 * (the tangent train's, up to 128, are not checked: it is consumed by the
 * caller). */
int tt_tangent_train(int d, const int64_t* dims, const int64_t* ranks, const double* const* U,
                     const double* const* V, const double* const* dC, double t_host, const double* t_dev,
                     int with_base, double* const* W, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TTUTV_H */
