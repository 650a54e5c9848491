// Internal declarations shared by the HIP translation units of libttutv.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stddef.h>
#include <stdint.h>

namespace ttutv {

// Kernel timing: while `timing.start` is set on the calling thread, the one
// kernel the next launcher enqueues carries the two events in its own
// dispatch (hipExtLaunchKernelGGL), so the events bracket exactly that kernel.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchTiming g_launch_timing;

#define TT_LAUNCH(kernel, grid, block, shm, st, ...)                                                  \
  do {                                                                                              \
    if (::ttutv::g_launch_timing.start)                                                             \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, st, ::ttutv::g_launch_timing.start,           \
                            ::ttutv::g_launch_timing.stop, 0, __VA_ARGS__);                         \
    else                                                                                            \
      hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                                \
  } while (0)

// Storage of a tall m x n matrix (m >= 1 rows on the long side, n columns on
// the core side).  ROW: element (i, j) at i*n + j (left-to-right sweep, where
// the tall matrix is the transpose of a column-major unfolding).  COL: at
// i + j*m (right-to-left sweep, the unfolding itself).
enum Layout : int { ROW = 0, COL = 1 };

constexpr int kCMax = 64;      // widest small side handled by the tall kernels
constexpr int kGramMax = 64;   // n up to which a step forms A^T A in one pass

// One record per step of the sweep, written on the device, read back once.
struct StepRec {
  double normC2;    // ||C||_F^2 of the factorised matrix
  double kept2;     // sum_{i<=r} s_i^2 (energy of the rank-r part)
  double carry2;    // ||carry||_F^2 as measured on the written carry
  double resid2;    // ||C - C_r||_F^2 measured directly (exact_delta), else -1
  double rho2;      // ||carry - fl32(carry)||_F^2 when the carry is stored in FP32
  double lam[kCMax];// squared singular values of the ell x ell triangle, descending
  int32_t r;        // rank chosen
  int32_t sat;      // eps rule met (1) / not met (0); 1 for fixed ranks
  int32_t ell;
  int32_t sweeps;   // Jacobi sweeps used by the Rayleigh-Ritz eigen-decomposition
};

// ---- tall streaming kernels (tt_tall.hip) --------------------------------
// Number of row chunks the A^T Y kernel uses for an m x n by m x c product.
int atb_chunks(int64_t m, int n, int c);
// partials[ch][j + n*cc] = sum over the rows of chunk ch of A(i,j) Y(i,cc).
hipError_t launch_atb(const void* A, int a_f32, const void* Y, int y_f32, int64_t m, int n,
                      int c, int layout, double* partials, int nchunks, hipStream_t st);
// Number of workgroups (and of sum-of-squares partials) the A*W kernel uses.
int ax_chunks(int64_t m, int n, int c);
hipError_t launch_ax(const void* A, int a_f32, const double* W, void* Y, int y_f32, int64_t m,
                     int n, int c, int layout, int nchunks, double* sumsqA, double* sumsqY,
                     double* rerr, hipStream_t st);
// Mixed-precision power-iteration products on FP32-accumulating matrix cores,
// operands rounded to BF16 (bf16 = 1) or kept FP32 (bf16 = 0).  Y (FP32,
// layout) = A W; partials[ch] = A^T Y over the rows of chunk ch (stored FP64),
// atb_lp_chunks(m, n) chunks.
hipError_t launch_ax_lp(const void* A, int a_f32, const double* W, float* Y, int64_t m, int n, int c, int layout,
                        int bf16, hipStream_t st);
int atb_lp_chunks(int64_t m, int n);
hipError_t launch_atb_lp(const void* A, int a_f32, const float* Y, int64_t m, int n, int c, int layout,
                         double* partials, int nchunks, int bf16, hipStream_t st);
// partials[ch] = A^T Y over the rows of chunk ch (n x c column-major, FP64) for
// any n: 128 columns of A per workgroup, row tiles prefetched into registers;
// FP64 matrix cores, or FP32 ones (f32_mma, FP32 data only).  atb2_chunks(m, n)
// chunks (never more than atb_chunks).
// Z = A^T (A X) in one pass over A (FP64, column-major A; see fused_ata_ok):
// fused_ata_blocks(m) partials of n x c (the count the launch takes), reduced
// with launch_reduce.
bool fused_ata_ok(int a_f32, int64_t m, int n, int c, int layout);
int fused_ata_blocks(int64_t m);
hipError_t launch_fused_ata(const double* A, const double* X, int64_t m, int n, int c, double* partials, int nblocks,
                            hipStream_t st);
int atb2_chunks(int64_t m, int n);
hipError_t launch_atb2(const void* A, int a_f32, const void* Y, int y_f32, int64_t m, int n, int c, int layout,
                       int f32_mma, double* partials, int nchunks, hipStream_t st);
// resid[ch] = sum over chunk rows of (A - Cr V1^T)^2, Cr m x r in `layout`, V1 n x r k-major.
int resid_chunks(int64_t m);
hipError_t launch_resid(const void* A, int a_f32, const void* Cr, int c_f32, const double* V1, int64_t m,
                        int n, int r, int layout, int nchunks, double* resid, hipStream_t st);
// out[e] (+ out2[e] if out2) = sum_ch partials[ch*size + e], fixed order.  With
// `stripes` (kReduceStripes * size doubles, not overlapping partials), many chunks
// of a short vector are summed in two stages: stripes of consecutive chunks in
// parallel, then the stripes in order.
constexpr int kReduceStripes = 64;
hipError_t launch_reduce(const double* partials, int nchunks, int64_t size, double* out,
                         double* out2, hipStream_t st, double* stripes = nullptr);

// ---- single-workgroup factorisations (tt_small.hip) -----------------------
struct SolveArgs {
  int n, ell, q;
  uint64_t seed;
  int label, n_mode, n_rank, mode_fastest;
  int r_fixed;            // > 0: fixed rank; <= 0: eps rule
  double eps_factor2;     // (w_k * eps)^2: eps_k^2 = eps_factor2 * ||A||^2
  int max_rank;
  int core_layout;        // 0: core = V1 column-major (L2R); 1: core = V1 row-major (R2L)
  double* core;           // core buffer (or NULL)
  double* V1;             // n x r, k-major (V1(i,c) at i*r + c)
  double* W;              // carry weights (non-Gram: ell x r, k-major)
  StepRec* rec;
  const double* normC2_src;  // NULL: take trace(H) (Gram mode, first step)
  double* normA2;            // ||A||^2 (written on the first step, read for eps_k)
  int first;
  // When set, ||C||^2 of this step is the previous carry's sum of squares still
  // held as nc_n per-workgroup partials: the solve sums them (fixed order) and
  // also stores the sum at nc_out (the previous step's record); normC2_src is
  // then not read.
  const double* nc_parts;
  int nc_n;
  double* nc_out;
};
// Gram mode (n <= kGramMax): H = A^T A (n x n column-major).
hipError_t launch_gram_solve(const double* H, const SolveArgs& a, hipStream_t st);
// Gaussian test matrix G (n x ell, k-major: G(i,j) at i*ell + j) of the step.
hipError_t launch_gen_sketch(double* G, const SolveArgs& a, hipStream_t st);
// X = orth(M): explicit orthonormal factor of the Householder QR of M (n x c,
// column-major; overwritten); X is written k-major.  Tall M is factorised as a
// tree of block QRs in `scratch` (orth_scratch(n, c) doubles, may be 0).
int64_t orth_scratch(int n, int c);
hipError_t launch_orth(double* M, double* X, int n, int c, double* scratch, int64_t scratch_len, hipStream_t st);
// X = orth(M) (M n x c column-major, X k-major) by shifted CholeskyQR3: three
// Gram / shifted Cholesky / triangular-solve rounds,
// scratch of orth_cholqr_scratch(n, c) doubles; M is not modified.
int64_t orth_cholqr_scratch(int n, int c);
hipError_t launch_orth_cholqr(const double* M, double* X, int n, int c, double* scratch, int64_t scratch_len,
                              hipStream_t st);
// Rayleigh-Ritz on span(X) (X k-major): K = (A X)^T (A X) (ell x ell) -> rank,
// V1 = X Z_r, W = Z_r.
hipError_t launch_rr_solve(const double* K, const double* X, const SolveArgs& a, hipStream_t st);
// Alg. 4 step, one round of the long-side orthonormalisation: T =
// P Lambda^{-1/2} (ell x ell, k-major) from K = Y^T Y = P Lambda P^T, so that
// Y T is orthonormal on the numerical span of Y.
hipError_t launch_alg4_basis(const double* K, double* T, int ell, hipStream_t st);
// Alg. 4 step, factorisation: from E = Bt^T Bt (ell x ell) and Bt = A^T U
// (n x ell column-major, U orthonormal): rank, core V1 = Bt W_r S_r^{-1},
// carry weights W_r S_r (ell x r k-major, carry = U W).
hipError_t launch_alg4_solve(const double* E, const double* Bt, const SolveArgs& a, hipStream_t st);

// ---- deflation inner kernel (tt_small.hip, tt_deflation.hip) ---------------
// One core-side vector at a time (the USV-plus reading of the paper's fastest
// TT-ULV variant): vector j starts from column j of the step's test matrix with
// the earlier vectors projected out (two classical Gram-Schmidt rounds), takes
// q power steps x <- P(A^T A x) / ||P(A^T A x)||, and adds ||A v_j||^2 to the
// kept energy; the search ends at the fixed rank, at the first j meeting the
// rank rule, or after cap vectors.
struct DeflState {
  double normC2;   // ||C||_F^2 of the step (from the first pass over A)
  double kept;     // sum of the energies of the vectors kept so far
  int32_t r;       // vectors kept
  int32_t sat;     // rank rule met (1 for fixed ranks)
  int32_t done;    // search ended: later launches of the step do nothing
  int32_t pad;
};
struct DeflArgs {
  SolveArgs a;     // n, q, generator, rank target, core / V1 / record outputs
  int cap;         // vectors at most (the fixed rank, or the eps-mode cap)
  double* V;       // n x cap, column j at V + j n
  double* x;       // the vector being iterated (n)
  DeflState* st;
};
// Gram mode (n <= kGramMax): the whole search on H = A^T A in one workgroup,
// then the core, V1 and the step record.
hipError_t launch_defl_gram(const double* H, const SolveArgs& a, int cap, hipStream_t st);
// Tall mode: zr = [z (n), ||A x||^2, ||A w||^2, ||A||_F^2] from one pass.
hipError_t launch_defl_start(const DeflArgs& d, hipStream_t st);
hipError_t launch_defl_update(const double* zr, const DeflArgs& d, int j, int has_w, int finish, int first_pass,
                              hipStream_t st);
hipError_t launch_defl_last(const double* zr, const DeflArgs& d, hipStream_t st);
hipError_t launch_defl_finish(const DeflArgs& d, hipStream_t st);
// The pass: per workgroup, z = A^T (A x) over its rows, ||A x||^2, ||A w||^2 and
// (want_sq) ||A||_F^2, into part[g * (n + 3) ..]; x and w may be NULL.
constexpr int kDeflMaxN = 4096;
int defl_pass_groups(int64_t m, int n, int layout);
// Doubles of scratch the passes of a step need for any core side up to n_max:
// the per-workgroup partials and the stripes of their reduction.
int64_t defl_pass_scratch(int64_t m, int n_max, int layout);
hipError_t launch_defl_pass(const void* A, int a_f32, int64_t m, int n, int layout, const double* x,
                            const double* w, int want_sq, double* part, int groups, hipStream_t st);

// ---- train contractions (tt_train.hip) ------------------------------------
// C (M x N) = A (M x K) B (K x N), all column-major, K <= kCMax; C is double or float.
hipError_t launch_gemm_smallk(const double* A, const double* B, void* C, int c_f32, int64_t M,
                              int64_t N, int K, hipStream_t st);
// C (M x N, column-major) = A B with A(m, k) at A[m sam + k sak] and B(k, n)
// at B[k sbk + n sbn]; the k range is split over `splits` workgroup layers
// (gemm_any_splits) whose M x N partials (partials: splits * M * N doubles,
// unused for one split) are summed in a fixed order.
int gemm_any_splits(int64_t M, int64_t N, int64_t K);
hipError_t launch_gemm_any(const double* A, int64_t sam, int64_t sak, const double* B, int64_t sbk, int64_t sbn,
                           double* C, int64_t M, int64_t N, int64_t K, double* partials, int splits, hipStream_t st);
// out (cols x rows) = in^T (in: rows x cols), both column-major.
hipError_t launch_transpose(const double* in, int64_t rows, int64_t cols, double* out, hipStream_t st);
hipError_t launch_sample(int d, const int64_t* dims, const int64_t* ranks,
                         const double* const* cores, const int64_t* idx, int64_t N, double* out,
                         hipStream_t st);
// One sample per thread (every rank <= 32: sample_rm > 0): cores FP64 or FP32
// (f32), staged in LDS when they fit.
int sample_rm(int d, const int64_t* ranks);
hipError_t launch_sample2(int d, const int64_t* dims, const int64_t* ranks, const void* const* cores, int f32,
                          const int64_t* idx, int64_t N, double* out, hipStream_t st);
// Backward through interface products stored in `work` and per-workgroup
// partial gradients summed in a fixed order; gcores in the cores' type.
size_t sample_bwd2_workspace(int d, const int64_t* dims, const int64_t* ranks, int64_t N);
hipError_t launch_sample_bwd2(int d, const int64_t* dims, const int64_t* ranks, const void* const* left,
                              const void* const* right, int f32, const int64_t* idx, int64_t N, const double* gout,
                              void* const* gcores, void* work, size_t work_bytes, hipStream_t st);
// right_cores: NULL for the gradient of the train itself; else the right
// interface products come from right_cores (a second form of the same train).
hipError_t launch_sample_bwd(int d, const int64_t* dims, const int64_t* ranks,
                             const double* const* cores, const double* const* right_cores, const int64_t* idx,
                             int64_t N, const double* gout, double* const* gcores, hipStream_t st);

// ---- carry pass that also forms the next step's first sketch (tt_carry_sketch.hip)
// H (I x n1 x c) = V1 G_i for every slab i; V1 (n1 x r) and G (I r x c) k-major.
hipError_t launch_sketch_fold(const double* V1, const double* G, double* H, int I, int n1, int r, int c,
                              hipStream_t st);
// Workgroups of the fused pass (<= 2048; one per-workgroup partial each).
int carry_sketch_groups(int64_t m2, int a_f32, int c_f32);
// Shapes and alignments the fused pass handles (column-major A of m2 I rows and n1
// columns, carry C of r columns, Y of m2 x c; FP64 carry and Y, or FP32 both).
bool carry_sketch_ok(const void* A, int a_f32, const void* C, int c_f32, const void* Y, int64_t m2, int I, int n1,
                     int r, int c);
// C = A V1 and Y = sum_i A_i H_i; sumsqC[b] (and rerr[b] for an FP32 carry) per workgroup.
hipError_t launch_carry_sketch(const void* A, int a_f32, int64_t m2, int I, int n1, const double* V1, int r,
                               const double* H, int c, void* C, int c_f32, void* Y, double* sumsqC, double* rerr,
                               int groups, hipStream_t st);

// ---- completion steps (tt_manifold.hip) ------------------------------------
size_t reduce_workspace_bytes();
hipError_t launch_residual(const double* pred, const double* vals, int64_t n, double* z, double* f, double* work,
                           hipStream_t st);
hipError_t launch_line_step(const double* p, const double* z, int64_t n, double* out3, double* work,
                            hipStream_t st);
hipError_t launch_axpy(int64_t n, double a, const double* a_dev, const double* x, double* y, hipStream_t st);
hipError_t launch_tangent_project(int d, const int64_t* dims, const int64_t* ranks, const double* const* U,
                                  const double* const* G, double* const* dC, hipStream_t st);
hipError_t launch_tangent_train(int d, const int64_t* dims, const int64_t* ranks, const double* const* U,
                                const double* const* V, const double* const* dC, double t, const double* t_dev,
                                int base, double* const* W, hipStream_t st);

}  // namespace ttutv
