// Diagonal-block kernels, one workgroup per block (kb <= 128).
//
// potrf_diag: Cholesky of the diagonal block, the "chol" step of section
// 3.3.1, and in the same sweep the inverse of the resulting triangle (needed
// by the panel solve L21 = A21 L11^-T, done as a product with the inverse as
// the paper does with its lower-triangular inverse, section 3.2): 16 x 16
// tiles held in registers and updated with matrix-core products, see
// diag_tile_factor_inverse.
//
// trtri_diag_batched: inverses of all diagonal blocks of a given factor, one
// workgroup per block held in LDS (128 x 129 doubles = 132 KB of the CU's
// 160 KB): the D^-1 of each step of the reverse sweep (3.3.2); block q goes
// to Dinv + q*b*b with leading dimension b.
#include "diag.hpp"

namespace gpc {
namespace {

constexpr int P = kDiagMax + 1;   // LDS row pitch (odd: spreads column walks over banks)

// X = L^-1 for the lower triangle L in S.  X[i][c] (i > c) is kept in the
// strict upper triangle at S[c][i], the diagonal of X in xd.  Row j of X is
// final once divided by L_jj; it is then subtracted, times L_ij, from every
// later row i (forward substitution on all columns at once).  The division of
// row j is deferred to step j+1, one barrier per step.
__device__ void invert_in_lds(double* S, double* xd, int kb)
{
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    for (int i = tid; i < kb; i += 256) xd[i] = 1.0;
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        if (c > r) S[r * P + c] = 0.0;
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        if (j > 0) {
            const double l = S[(j - 1) * P + (j - 1)];
            for (int c = tid; c < j; c += 256) {
                if (c == j - 1) xd[j - 1] /= l;
                else S[c * P + (j - 1)] /= l;
            }
        }
        const double ljj = S[j * P + j];
        const int m = kb - j - 1;
        for (int q = tx; q <= j; q += 16) {
            const double xjc = (q == j ? xd[j] : S[q * P + j]) / ljj;
            for (int p = ty; p < m; p += 16) {
                const int i = j + 1 + p;
                S[q * P + i] -= S[i * P + j] * xjc;
            }
        }
        __syncthreads();
    }
    {
        const double l = S[(kb - 1) * P + (kb - 1)];
        for (int c = tid; c < kb; c += 256) {
            if (c == kb - 1) xd[kb - 1] /= l;
            else S[c * P + (kb - 1)] /= l;
        }
    }
    __syncthreads();
}

// NT: 16 x 16 tile rows of the block (blocks up to 16 NT; smaller blocks take
// the smaller instance).  At most 256 registers per lane, so that the kernel
// fits on a CU beside a product kernel's workgroup.
template <int NT>
__global__ void __launch_bounds__(256, 2)
potrf_tile_kernel(int kb, double* A, int64_t lda, double* Linv, int64_t ldi, int32_t* info, int64_t col0)
{
    __shared__ double F[NT * 256], LU[256];
    diag_tile_factor_inverse<NT>(kb, A, lda, Linv, ldi, info, col0, F, LU);
}

__global__ void __launch_bounds__(256)
trtri_batched_kernel(int64_t n, int b, const double* L, int64_t ldl, double* Dinv)
{
    __shared__ double S[kDiagMax * P];
    __shared__ double xd[kDiagMax];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * b;
    const int kb = (int)min((int64_t)b, n - r0);
    const double* D = L + r0 * ldl + r0;
    double* X = Dinv + (int64_t)blockIdx.x * b * b;
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        S[r * P + c] = c <= r ? D[r * ldl + c] : 0.0;
    }
    __syncthreads();
    invert_in_lds(S, xd, kb);
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        X[r * b + c] = c < r ? S[c * P + r] : (c == r ? xd[r] : 0.0);
    }
}

__global__ void __launch_bounds__(256)
trtri_pairs_kernel(int64_t n, const double* L, int64_t ldl, double* Dinv)
{
    __shared__ double S[kDiagMax * P];
    __shared__ double xd[kDiagMax];
    const int tid = threadIdx.x;
    const int64_t p = blockIdx.x;
    const int64_t r0 = p * kDiagMax;
    const int kb = (int)min((int64_t)kDiagMax, n - r0);
    const double* D = L + r0 * ldl + r0;
    double* X = Dinv + (p >> 1) * (2 * kDiagMax) * (2 * kDiagMax) + (p & 1) * (kDiagMax * 2 * kDiagMax + kDiagMax);
    const int64_t ldx = 2 * kDiagMax;
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        S[r * P + c] = c <= r ? D[r * ldl + c] : 0.0;
    }
    __syncthreads();
    invert_in_lds(S, xd, kb);
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        X[r * ldx + c] = c < r ? S[c * P + r] : (c == r ? xd[r] : 0.0);
    }
}

__global__ void fill_f64_kernel(int64_t count, double* p, double v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = v;
}

}  // namespace

hipError_t trtri_diag_pairs(hipStream_t s, int64_t n, const double* L, int64_t ldl, double* Dinv)
{
    if (n <= 0) return hipSuccess;
    const int64_t nsub = (n + kDiagMax - 1) / kDiagMax;
    hipLaunchKernelGGL(trtri_pairs_kernel, dim3((unsigned)nsub), dim3(256), 0, s, n, L, ldl, Dinv);
    return hipGetLastError();
}

hipError_t fill_f64(hipStream_t s, int64_t count, double* p, double v)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, p, v);
    return hipGetLastError();
}

hipError_t potrf_diag(hipStream_t s, int kb, double* A, int64_t lda, double* Linv, int64_t ldi,
                      int32_t* info, int64_t col0)
{
    if (kb <= 0) return hipSuccess;
    if (kb > kDiagMax || lda > (int64_t(1) << 20)) return hipErrorInvalidValue;   // 31-bit row-band offsets
    if (kb <= 32)
        hipLaunchKernelGGL(potrf_tile_kernel<2>, dim3(1), dim3(256), 0, s, kb, A, lda, Linv, ldi, info, col0);
    else if (kb <= 64)
        hipLaunchKernelGGL(potrf_tile_kernel<4>, dim3(1), dim3(256), 0, s, kb, A, lda, Linv, ldi, info, col0);
    else
        hipLaunchKernelGGL(potrf_tile_kernel<kDiagMax / 16>, dim3(1), dim3(256), 0, s, kb, A, lda, Linv, ldi, info,
                           col0);
    return hipGetLastError();
}

hipError_t trtri_diag_batched(hipStream_t s, int64_t n, int b, const double* L, int64_t ldl, double* Dinv)
{
    if (n <= 0) return hipSuccess;
    if (b <= 0 || b > kDiagMax) return hipErrorInvalidValue;
    const int64_t nblk = (n + b - 1) / b;
    hipLaunchKernelGGL(trtri_batched_kernel, dim3((unsigned)nblk), dim3(256), 0, s, n, b, L, ldl, Dinv);
    return hipGetLastError();
}

}  // namespace gpc
