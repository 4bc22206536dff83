// Memory-bound helpers of the blocked factor and reverse sweep: flag reset,
// zeroing of the strict upper triangle (outputs are lower-triangular views,
// section 2.2), and the fixed-order sums of split-K partial products
// (section 3.1, "large k": s partial copies added by a separate kernel; here
// the copies are added in increasing order so results do not depend on timing).
#include "internal.hpp"

namespace gpc {
namespace {

__global__ void fill_i32_kernel(int32_t* p, int32_t v) { *p = v; }

// One workgroup per 64 x 64 tile on or above the diagonal (tile index in
// the row-by-row enumeration of that triangle of tiles); elements with
// column > row are zeroed.
__global__ void zero_upper_kernel(int64_t n, double* A, int64_t lda)
{
    const int64_t b = blockIdx.x;
    int64_t t = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (t * (t + 1) / 2 > b) --t;
    while ((t + 1) * (t + 2) / 2 <= b) ++t;
    const int64_t r0 = (b - t * (t + 1) / 2) * 64, c0 = t * 64;   // tile row <= tile column
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int64_t r = r0 + e / 64, c = c0 + e % 64;
        if (r < n && c < n && c > r) A[r * lda + c] = 0.0;
    }
}

__global__ void convert_lower_kernel(int64_t n, const double* L, int64_t ldl, float* Lf, int64_t ldf)
{
    const int64_t r = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6);
    const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (r < n && c < r) Lf[r * ldf + c] = (float)L[r * ldl + c];
}

// sum_{z<S} p[z * pstride] with z increasing, the loads issued sixteen at a
// time (the additions keep that order, so the result does not depend on the
// batching).
__device__ __forceinline__ double slice_sum(const double* p, int S, int64_t pstride)
{
    constexpr int G = 16;
    double s = 0.0;
    for (int z = 0; z < S; z += G) {
        double v[G];
#pragma unroll
        for (int k = 0; k < G; ++k) v[k] = z + k < S ? p[(int64_t)(z + k) * pstride] : 0.0;
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (z + k < S) s += v[k];
    }
    return s;
}

__global__ void reduce_sub_kernel(int64_t M, int64_t N, const double* P, int S, int64_t pstride,
                                  double* C, int64_t ldc)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * N) return;
    const int64_t m = e / N, n = e % N;
    C[m * ldc + n] -= slice_sum(P + m * N + n, S, pstride);
}

__global__ void reduce_tril_kernel(int b, const double* D, int64_t ldd, const double* P, int S,
                                   int64_t pstride, double* W)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= b * b) return;
    const int m = e / b, n = e % b;
    double v = 0.0;
    if (m >= n) v = D[m * ldd + n] - slice_sum(P + (int64_t)m * b + n, S, pstride);
    W[e] = v;
}

// Element (r, c) of a b x b sum v = sum_z P[z][r][c] (P: b x b slices,
// slice stride pstride) stored with the epilogue of mode: 0 C[r][c] = C[c][r]
// = v for r >= c; 1 C[c][r] = v; 2 C[r][c] = v, Cf[r][c] = (float)v if Cf,
// C2[r][c] = r > c ? v : r == c ? v / 2 : 0.
__global__ void reduce_epi_kernel(int b, const double* P, int S, int64_t pstride, int mode, double* C, int64_t ldc,
                                  float* Cf, int64_t ldcf, double* C2, int64_t ldc2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= b * b) return;
    const int r = e / b, c = e % b;
    if (mode == 0 && r < c) return;
    const double v = slice_sum(P + e, S, pstride);
    if (mode == 0) {
        C[(int64_t)r * ldc + c] = v;
        C[(int64_t)c * ldc + r] = v;
    } else if (mode == 1) {
        C[(int64_t)c * ldc + r] = v;
    } else {
        C[(int64_t)r * ldc + c] = v;
        if (Cf) Cf[(int64_t)r * ldcf + c] = (float)v;
        C2[(int64_t)r * ldc2 + c] = r > c ? v : (r == c ? 0.5 * v : 0.0);
    }
}

}  // namespace

hipError_t reduce_epi(hipStream_t s, int b, const double* P, int S, int64_t pstride, int mode, double* C,
                      int64_t ldc, float* Cf, int64_t ldcf, double* C2, int64_t ldc2)
{
    if (b <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_epi_kernel, dim3((unsigned)((b * b + 255) / 256)), dim3(256), 0, s, b, P, S, pstride,
                       mode, C, ldc, Cf, ldcf, C2, ldc2);
    return hipGetLastError();
}

hipError_t fill_i32(hipStream_t s, int32_t* p, int32_t v)
{
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

hipError_t zero_strict_upper(hipStream_t s, int64_t n, double* A, int64_t lda)
{
    if (n <= 1) return hipSuccess;
    const int64_t t = (n + 63) / 64;
    hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)(t * (t + 1) / 2)), dim3(256), 0, s, n, A, lda);
    return hipGetLastError();
}

hipError_t convert_lower_f32(hipStream_t s, int64_t n, const double* L, int64_t ldl, float* Lf, int64_t ldf)
{
    if (n <= 1) return hipSuccess;
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((n + 3) / 4));
    hipLaunchKernelGGL(convert_lower_kernel, grid, dim3(256), 0, s, n, L, ldl, Lf, ldf);
    return hipGetLastError();
}

hipError_t reduce_sub(hipStream_t s, int64_t M, int64_t N, const double* P, int S, int64_t pstride,
                      double* C, int64_t ldc)
{
    if (M <= 0 || N <= 0 || S <= 0) return hipSuccess;
    const int64_t tot = M * N;
    hipLaunchKernelGGL(reduce_sub_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       M, N, P, S, pstride, C, ldc);
    return hipGetLastError();
}

hipError_t reduce_tril(hipStream_t s, int b, const double* D, int64_t ldd, const double* P, int S,
                       int64_t pstride, double* W)
{
    if (b <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_tril_kernel, dim3((unsigned)((b * b + 255) / 256)), dim3(256), 0, s,
                       b, D, ldd, P, S, pstride, W);
    return hipGetLastError();
}

}  // namespace gpc
