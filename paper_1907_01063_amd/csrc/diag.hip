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
// 160 KB), the inverse in registers (diag_inverse): the D^-1 of each step of
// the reverse sweep (3.3.2); block q goes to Dinv + q*b*b with leading
// dimension b.
#include "diag.hpp"

namespace gpc {
namespace {

// NT: 16 x 16 tile rows of the block (blocks up to 16 NT; smaller blocks take
// the smaller instance).  At most 256 registers per lane, so that the kernel
// fits on a CU beside a product kernel's workgroup.
template <int NT>
__global__ void __launch_bounds__(256, 2)
potrf_tile_kernel(int kb, double* A, int64_t lda, double* Linv, int64_t ldi, int32_t* info, int64_t col0, int prio)
{
    if (prio) __builtin_amdgcn_s_setprio(3);
    __shared__ double F[NT * 256], LU[256];
    diag_tile_factor_inverse<NT>(kb, A, lda, Linv, ldi, info, col0, F, LU);
}

// Inverse of diagonal block blockIdx.x (edge b <= kDiagMax) to
// Dinv + blockIdx.x * b * b, leading dimension b.
__global__ void __launch_bounds__(256)
trtri_batched_kernel(int64_t n, int b, const double* L, int64_t ldl, double* Dinv)
{
    __shared__ double Ls[kDiagMax * (kDiagMax + 1)];
    __shared__ double rowbuf[kDiagMax];
    const int64_t r0 = (int64_t)blockIdx.x * b;
    const int kb = (int)min((int64_t)b, n - r0);
    diag_inverse<kDiagMax / 16>(kb, L + r0 * ldl + r0, ldl, Dinv + (int64_t)blockIdx.x * b * b, b, Ls, rowbuf);
}

// Inverse of the kDiagMax-block p = blockIdx.x into the diagonal of the
// b-block p / (b / kDiagMax) of Dinv (leading dimension b), at its
// (p mod (b / kDiagMax))-th kDiagMax position.
__global__ void __launch_bounds__(256)
trtri_into_kernel(int64_t n, int b, const double* L, int64_t ldl, double* Dinv)
{
    __shared__ double Ls[kDiagMax * (kDiagMax + 1)];
    __shared__ double rowbuf[kDiagMax];
    const int64_t p = blockIdx.x;
    const int64_t r0 = p * kDiagMax;
    const int kb = (int)min((int64_t)kDiagMax, n - r0);
    const int per = b / kDiagMax;
    double* X = Dinv + (p / per) * (int64_t)b * b + (p % per) * ((int64_t)kDiagMax * b + kDiagMax);
    diag_inverse<kDiagMax / 16>(kb, L + r0 * ldl + r0, ldl, X, b, Ls, rowbuf);
}

__global__ void fill_f64_kernel(int64_t count, double* p, double v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = v;
}

}  // namespace

hipError_t trtri_diag_into(hipStream_t s, int64_t n, int b, const double* L, int64_t ldl, double* Dinv)
{
    if (n <= 0) return hipSuccess;
    if (b < kDiagMax || b % kDiagMax != 0) return hipErrorInvalidValue;
    const int64_t nsub = (n + kDiagMax - 1) / kDiagMax;
    hipLaunchKernelGGL(trtri_into_kernel, dim3((unsigned)nsub), dim3(256), 0, s, n, b, L, ldl, Dinv);
    return hipGetLastError();
}

hipError_t fill_f64(hipStream_t s, int64_t count, double* p, double v)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, p, v);
    return hipGetLastError();
}

hipError_t potrf_diag(hipStream_t s, int kb, double* A, int64_t lda, double* Linv, int64_t ldi,
                      int32_t* info, int64_t col0, int prio)
{
    if (kb <= 0) return hipSuccess;
    if (kb > kDiagMax || lda > (int64_t(1) << 20)) return hipErrorInvalidValue;   // 31-bit row-band offsets
    if (kb <= 32)
        hipLaunchKernelGGL(potrf_tile_kernel<2>, dim3(1), dim3(256), 0, s, kb, A, lda, Linv, ldi, info, col0, prio);
    else if (kb <= 64)
        hipLaunchKernelGGL(potrf_tile_kernel<4>, dim3(1), dim3(256), 0, s, kb, A, lda, Linv, ldi, info, col0, prio);
    else
        hipLaunchKernelGGL(potrf_tile_kernel<kDiagMax / 16>, dim3(1), dim3(256), 0, s, kb, A, lda, Linv, ldi, info,
                           col0, prio);
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
