// Internal declarations shared by the HIP translation units of libgpchol.
// Row-major storage throughout: element (i, j) of X is X[i * ld + j].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpc {

// Largest diagonal block handled inside one workgroup's LDS.
constexpr int kDiagMax = 128;
// Largest input dimension of the GP covariance kernels.
constexpr int kMaxGpDim = 16;

// ---- GEMM on MFMA ---------------------------------------------------------
// acc[m][n] = sum_{k in [k0,k1)} Aop[m][k] * Bop[k][n], then an epilogue.
//   A layout  MK: Aop[m][k] = A[m*lda + k]      KM: Aop[m][k] = A[k*lda + m]
//   B layout  KN: Bop[k][n] = B[k*ldb + n]      NK: Bop[k][n] = B[n*ldb + k]
// For layout KM the first `head_k` values of k may come from a separate
// matrix `Ahead` (row k of Ahead, leading dimension ldah); k >= head_k then
// reads row (k - head_k) of A.
enum Epi : int {
    EPI_SUB = 0,      // C[m][n] -= acc
    EPI_STORE = 1,    // C[m][n]  = acc   (C may alias A when one tile spans all N)
    EPI_PARTIAL = 2,  // C[z*pstride + m*ldc + n] = acc   (split-K slice z)
    EPI_SYMLOW = 3,   // for m >= n: C[m][n] = C[n][m] = acc   (symmetric from lower)
    EPI_PHI = 4,      // C[m][n] = acc (full);  C2[m][n] = m>n ? acc : m==n ? acc/2 : 0
    EPI_ADD = 5       // C[m][n] += acc
};

struct GemmArgs {
    int64_t M, N, K;
    const void* A; int64_t lda;
    const void* B; int64_t ldb;
    double* C; int64_t ldc;
    double* C2; int64_t ldc2;
    const void* Ahead; int64_t ldah; int64_t head_k;
    int64_t kchunk;     // split-K chunk (multiple of the kernel's BK); splits = gridDim.z
    int64_t pstride;    // EPI_PARTIAL slice stride (elements)
    int32_t a_lower;    // nonzero: A is lower-triangular as stored; its strict upper is never read
    float* Cf; int64_t ldcf;  // EPI_STORE / EPI_PHI: optional FP32 copy of the stored C (nullptr = none)
    int32_t c_lower;          // nonzero: never write C elements with col > row (C-local indices)
    int64_t bsA, bsB, bsC;    // batch strides (elements) applied per blockIdx.y
    int32_t negate;           // EPI_STORE: store -acc
    int32_t group;            // tile order: bands of `group` tile rows (0/1 = row by row); set by the launcher
    int64_t kstep;            // > 0: output rows m use only k < (m / kstep + 1) kstep (a staircase);
                              // kstep a multiple of the tile height
    int32_t prio;             // nonzero: the waves raise their issue priority (s_setprio): a launch on
                              // the critical path beside a long product
};

// TILE_64W: 64 x 128 tiles of 8 waves (twice the workgroups of TILE_128 for
// the in-place panel products, whose one tile column must span all N)
enum TileCfg : int { TILE_128 = 0, TILE_64 = 1, TILE_64W = 2 };

// Launchers (hipError_t from the launch).  `lower_tiles`: M == N and only tiles
// on or below the diagonal are computed, and only elements with m >= n written.
hipError_t gemm_f64(hipStream_t s, TileCfg cfg, bool a_km, bool b_nk, Epi epi,
                    bool lower_tiles, const GemmArgs& g, int splits, int batch = 1);
hipError_t gemm_f32in(hipStream_t s, TileCfg cfg, bool a_km, bool b_nk, Epi epi,
                      bool lower_tiles, const GemmArgs& g, int splits, int batch = 1);

// ---- diagonal blocks (single workgroup each) ------------------------------
// Factor the kb x kb diagonal block at A (in place, upper zeroed), write its
// inverse (lower, kb x kb, leading dimension ldi, upper zeroed) to Linv, and
// record the first failing pivot as info = col0 + j + 1 if info is still 0.
hipError_t potrf_diag(hipStream_t s, int kb, double* A, int64_t lda, double* Linv,
                      int64_t ldi, int32_t* info, int64_t col0, int prio = 0);
// Inverses of the diagonal blocks of L: block q covers rows/cols [q*b, min(n,(q+1)*b)),
// its inverse goes to Dinv + q*b*b (leading dimension b, upper zeroed).
hipError_t trtri_diag_batched(hipStream_t s, int64_t n, int b, const double* L, int64_t ldl,
                              double* Dinv);
// Inverses of the 128-blocks of L written onto the diagonals of b-blocks (b a
// multiple of 128): sub-block p goes to Dinv + (p/per)*b*b + (p%per)*(128*b+128),
// per = b/128, leading dimension b (the rest of each b-block is left untouched).
hipError_t trtri_diag_into(hipStream_t s, int64_t n, int b, const double* L, int64_t ldl, double* Dinv);
hipError_t fill_f64(hipStream_t s, int64_t count, double* p, double v);
// Inverses of the b x b diagonal blocks of L (b <= 128, or b = 256 or 512
// composed level by level from 128-block inverses), lower with zero strict
// upper, at Dinv + q*b*b.  Tmp: ceil(n/b) * (b/2)^2 doubles of scratch (b > 128).
hipError_t diag_block_inverses(hipStream_t s, int64_t n, int b, const double* L, int64_t ldl, double* Dinv,
                               double* Tmp);

// ---- elementwise helpers ---------------------------------------------------
// Lf[i][j] = (float)L[i][j] for j < i (strict lower triangle only).
hipError_t convert_lower_f32(hipStream_t s, int64_t n, const double* L, int64_t ldl, float* Lf, int64_t ldf);
hipError_t fill_i32(hipStream_t s, int32_t* p, int32_t v);
hipError_t zero_strict_upper(hipStream_t s, int64_t n, double* A, int64_t lda);
// C[m][n] -= sum_{z<S} P[z*pstride + m*N + n], z increasing.
hipError_t reduce_sub(hipStream_t s, int64_t M, int64_t N, const double* P, int S,
                      int64_t pstride, double* C, int64_t ldc);
// W[m][n] = m >= n ? D[m][n] - sum_z P[z][m][n] : 0   (b x b, W leading dim b)
// b x b split-K sums (slices of P, stride pstride, z increasing) stored with an
// epilogue: mode 0 symmetric from the lower triangle (C[r][c] = C[c][r]),
// 1 transposed (C[c][r]), 2 as EPI_PHI (C, optional FP32 copy Cf, C2 = phi).
hipError_t reduce_epi(hipStream_t s, int b, const double* P, int S, int64_t pstride, int mode, double* C,
                      int64_t ldc, float* Cf, int64_t ldcf, double* C2, int64_t ldc2);
hipError_t reduce_tril(hipStream_t s, int b, const double* D, int64_t ldd, const double* P,
                       int S, int64_t pstride, double* W);

// ---- solves and log-determinant --------------------------------------------
// Coupling blocks of the solves (b x b each at C + q*b*b, from the diagonal
// block inverses Dinv of trtri_diag_batched): trans 0: Cf_q = Dinv_q L_{q,q-1}
// (q >= 1); trans 1: Cb_q = L_{q+1,q} Dinv_q (q <= nblk-2).
hipError_t trsm_couplings(hipStream_t s, int trans, int64_t n, const double* L, int64_t ldl,
                          const double* Dinv, int b, double* C);
// B <- L^-1 B (trans 0) or L^-T B (trans 1) by block steps with Dinv and the
// couplings of the same direction (block b = 128 or 256): one launch for a
// single right-hand side (cus: compute units, sizes its grid; fail: start it
// with its error flag raised; rec: device word set to 1 if the sweep fails,
// never cleared here), else one launch per block step and group of
// right-hand sides.  Y: workspace of trsm_workspace(n) doubles.
int64_t trsm_workspace(int64_t n);
hipError_t trsm_blocked(hipStream_t s, int trans, int64_t n, int64_t nrhs, const double* L,
                        int64_t ldl, const double* Dinv, const double* Cpl, int b, double* B, int64_t ldb,
                        double* Y, int cus, int fail, uint32_t* rec);
// *out = 2 * sum_i log L_ii (fixed summation order).
hipError_t logdet(hipStream_t s, int64_t n, const double* L, int64_t ldl, double* out);

// ---- GP pieces and refinement (gp.hip) -------------------------------------
// theta (device): (s2, l_1..l_d, sn2).  K, Lbar: lower + zero upper written.
hipError_t gp_kgen_se(hipStream_t s, int64_t n, int d, const double* X, const double* theta, double* K, int64_t ldk);
hipError_t gp_lbar(hipStream_t s, int64_t n, const double* L, int64_t ldl, const double* alpha, const double* z,
                   double* Lbar, int64_t ldlb);
int64_t gp_hypergrad_parts(int64_t n, int d);   // doubles of workspace for gp_hypergrad_se
hipError_t gp_hypergrad_se(hipStream_t s, int64_t n, int d, const double* X, const double* theta, const double* Ab,
                           int64_t ldab, const double* scale, double* grad, double* part);
hipError_t gp_value(hipStream_t s, int64_t n, const double* z, const double* logdet, double* f);
// f = -1/2 a^T b - 1/2 logdet (fixed-order sum)
hipError_t gp_value_dot(hipStream_t s, int64_t n, const double* a, const double* b, const double* logdet, double* f);
int64_t symv_parts(int64_t n);                  // doubles of workspace for symv_lower
// out = y + sgn * K x  (K symmetric from its lower triangle; absk: |K|; x null: ones; y null: 0)
hipError_t symv_lower(hipStream_t s, int64_t n, const double* K, int64_t ldk, const double* x, int absk,
                      const double* y, double sgn, double* out, double* part);
// The same with x given, and in the same pass rowabs = |K| times ones (the row
// sums of |K|); part: 2 symv_parts(n) doubles.
hipError_t symv_lower_abs(hipStream_t s, int64_t n, const double* K, int64_t ldk, const double* x, const double* y,
                          double sgn, double* out, double* rowabs, double* part);
hipError_t refine_eta(hipStream_t s, int64_t n, const double* r, const double* x, const double* y,
                      const double* rowabs, double* eta);
hipError_t vec_axpy(hipStream_t s, int64_t n, const double* d, double* x);
hipError_t vec_copy(hipStream_t s, int64_t n, const double* a, double* b);
hipError_t vec_zero(hipStream_t s, int64_t n, double* a);

// ---- operations beside the Cholesky path (ops.hip) ---------------------------
// X = L^-1 (lower, strict upper zeroed; X must not overlap L): inverses of the
// 128-blocks, then the divide-and-conquer levels C3 = -C2 A3 C1 of section 3.2.
hipError_t trtri_full(hipStream_t s, int64_t n, const double* L, int64_t ldl, double* X, int64_t ldx);
// Split-K plan of a product of `tiles` 128 x 128 output tiles with inner
// dimension K on `slots` co-resident workgroups: splits (<= max_splits) and
// the chunk of k per split (a multiple of 32).
void plan_split_k(int64_t tiles, int64_t K, int max_splits, int64_t slots, int* splits, int64_t* chunk);
// C = op(A) op(B) + beta C (beta 0 or 1; op = transpose when ta / tb):
// 128 x 128 MFMA tiles, split along k when the plan says so (partial slices
// in ws, gemm_general_workspace doubles, then a fixed-order sum).
constexpr int kGemmMaxSplits = 32;
int64_t gemm_general_workspace(int64_t M, int64_t N, int64_t K, int cus, int max_splits);
hipError_t gemm_general(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, const double* A,
                        int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* ws,
                        int cus, int max_splits, int* splits_out);
// C[m][n] = beta C[m][n] + sum_{z<S} P[z*pstride + m*N + n] (z increasing), beta 0 or 1.
hipError_t reduce_store(hipStream_t s, int64_t M, int64_t N, const double* P, int S, int64_t pstride, double beta,
                        double* C, int64_t ldc);
// Bernoulli-logit GLM (y 0/1): lp, dalpha, dbeta (device) and dX (optional);
// ws: glm_workspace(n, k) doubles.  Rows are fused in one pass for
// k <= kGlmFusedMaxK, two passes beyond.
constexpr int64_t kGlmFusedMaxK = 2048;
int64_t glm_groups(int64_t n, int64_t k);
int64_t glm_workspace(int64_t n, int64_t k);
hipError_t glm_bernoulli_logit(hipStream_t s, int64_t n, int64_t k, const double* X, int64_t ldx, const int32_t* y,
                               const double* alpha, const double* beta, double* lp, double* dalpha, double* dbeta,
                               double* dX, int64_t lddx, double* ws);

// ---- batched persistent path (batched.hip) ----------------------------------
struct BatchTask {
    int32_t n;      // matrix order
    int32_t block;  // inner block (<= batched_max_block())
    int32_t idx;    // position in the caller's arrays (info index)
    int32_t pad;
    int64_t off;    // element offset of the matrix (row-major, leading dimension n)
};
int batched_max_block();
int64_t batched_scratch_doubles(int wgs);
// mode: 1 = factor, 2 = adjoint (Abase holds L), 3 = both.  counter: one device
// int32 reset by a kernel at the start (capturable).
hipError_t batched_launch(hipStream_t s, int nb, const BatchTask* tasks, double* Abase, double* Lbbase,
                          int32_t* info, int32_t* counter, double* ws, int wgs, int mode);
hipError_t spd_test_fill(hipStream_t s, int64_t n, double* A, double* Lb, int64_t off);

// Grouped schedule of the batched calls (grouped.hip): every block step one
// launch over all members.  prepare allocates and uploads the descriptors
// (synchronous); enqueue records the launches on a stream; free releases.
struct GroupedSchedule;
GroupedSchedule* grouped_prepare(int nb, const BatchTask* tasks, double* Abase, double* Lbbase, int32_t* info,
                                 int mode, hipError_t* err);
hipError_t grouped_enqueue(const GroupedSchedule* g, hipStream_t s, hipStream_t side, int32_t* info);
void grouped_free(GroupedSchedule* g);

}  // namespace gpc
