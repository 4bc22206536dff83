// Triangular solves with the factor and the log-determinant (the pieces a GP
// log-density needs: z = L^-1 y, alpha = L^-T z, log|K| = 2 sum log L_ii).
//
// The solves sweep the diagonal blocks of L (section 3.2 solves A x = b
// through the inverse of the triangle; here only the b x b diagonal blocks are
// inverted, and the off-diagonal blocks are applied as matrix-vector updates).
// One launch per block step: every workgroup recomputes the step's small
// product z_q = D_q^-1 y_q (or D_q^-T y_q) from the running right-hand side,
// workgroup 0 stores it, and each workgroup applies it to its own rows of the
// remaining right-hand side.  The running right-hand side lives in a separate
// workspace so that no workgroup reads what another one writes in the step.
// All are memory-bound matrix-vector work; reductions use fixed shuffle trees.
#include <algorithm>

#include "internal.hpp"

namespace gpc {
namespace {

constexpr int kRhsGroup = 8;   // right-hand sides handled per launch

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Forward step q: rows [j, j+bq) hold y_q in Y; z_q = Dinv_q y_q goes to B
// (block 0) and Y[r] -= L[r, j:j+bq] z_q for r in [j+bq, n).
__global__ void __launch_bounds__(256)
trsv_fwd_step(int64_t n, int nr, int64_t j, int bq, const double* L, int64_t ldl,
              const double* Dq, int b, double* Y, int64_t ldy, double* B, int64_t ldb,
              int64_t rows_per_block)
{
    __shared__ double z[kDiagMax][kRhsGroup];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = wave; i < bq; i += 4) {
        for (int c = 0; c < nr; ++c) {
            double p = 0.0;
            for (int t = lane; t <= i; t += 64) p += Dq[(int64_t)i * b + t] * Y[(j + t) * ldy + c];
            p = wave_sum(p);
            if (lane == 0) z[i][c] = p;
        }
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int e = threadIdx.x; e < bq * nr; e += 256) B[(j + e / nr) * ldb + e % nr] = z[e / nr][e % nr];
    const int64_t r0 = j + bq + (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    for (int64_t r = r0 + wave; r < r1; r += 4) {
        const double* lr = L + r * ldl + j;
        for (int c = 0; c < nr; ++c) {
            double p = 0.0;
            for (int t = lane; t < bq; t += 64) p += lr[t] * z[t][c];
            p = wave_sum(p);
            if (lane == 0) Y[r * ldy + c] -= p;
        }
    }
}

// Backward step q: z_q = Dinv_q^T y_q, then Y[r] -= sum_t L[j+t][r] z_q[t]
// for r in [0, j).  Threads walk r (contiguous within a row of L).
__global__ void __launch_bounds__(256)
trsv_bwd_step(int nr, int64_t j, int bq, const double* L, int64_t ldl, const double* Dq, int b,
              double* Y, int64_t ldy, double* B, int64_t ldb)
{
    __shared__ double z[kDiagMax][kRhsGroup];
    for (int e = threadIdx.x; e < bq * nr; e += 256) {
        const int i = e / nr, c = e % nr;
        double p = 0.0;
        for (int t = i; t < bq; ++t) p += Dq[(int64_t)t * b + i] * Y[(j + t) * ldy + c];
        z[i][c] = p;
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int e = threadIdx.x; e < bq * nr; e += 256) B[(j + e / nr) * ldb + e % nr] = z[e / nr][e % nr];
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= j) return;
    double acc[kRhsGroup];
    for (int c = 0; c < nr; ++c) acc[c] = 0.0;
    for (int t = 0; t < bq; ++t) {
        const double l = L[(j + t) * ldl + r];
        for (int c = 0; c < nr; ++c) acc[c] += l * z[t][c];
    }
    for (int c = 0; c < nr; ++c) Y[r * ldy + c] -= acc[c];
}

__global__ void copy_cols(int64_t n, int nr, const double* B, int64_t ldb, double* Y, int64_t ldy)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n * nr) Y[(e / nr) * ldy + e % nr] = B[(e / nr) * ldb + e % nr];
}

// One workgroup: thread t sums log L_ii over i = t, t+256, ... in increasing
// order, then a fixed binary tree combines the 256 partial sums.
__global__ void __launch_bounds__(256) logdet_kernel(int64_t n, const double* L, int64_t ldl, double* out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += log(L[i * ldl + i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = 2.0 * red[0];
}

}  // namespace

hipError_t trsm_blocked(hipStream_t s, int trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                        const double* Dinv, int b, double* B, int64_t ldb, double* Y)
{
    const int64_t nblk = (n + b - 1) / b;
    for (int64_t c0 = 0; c0 < nrhs; c0 += kRhsGroup) {
        const int nr = (int)std::min<int64_t>(kRhsGroup, nrhs - c0);
        double* Bc = B + c0;
        hipLaunchKernelGGL(copy_cols, dim3((unsigned)((n * nr + 255) / 256)), dim3(256), 0, s, n, nr, Bc, ldb, Y,
                           (int64_t)kRhsGroup);
        if (!trans) {
            for (int64_t q = 0; q < nblk; ++q) {
                const int64_t j = q * b;
                const int bq = (int)std::min<int64_t>(b, n - j);
                const int64_t rest = n - j - bq;
                const int64_t rpb = 64;
                const int64_t blocks = std::max<int64_t>(1, (rest + rpb - 1) / rpb);
                hipLaunchKernelGGL(trsv_fwd_step, dim3((unsigned)blocks), dim3(256), 0, s, n, nr, j, bq, L, ldl,
                                   Dinv + q * (int64_t)b * b, b, Y, (int64_t)kRhsGroup, Bc, ldb, rpb);
            }
        } else {
            for (int64_t q = nblk - 1; q >= 0; --q) {
                const int64_t j = q * b;
                const int bq = (int)std::min<int64_t>(b, n - j);
                const int64_t blocks = std::max<int64_t>(1, (j + 255) / 256);
                hipLaunchKernelGGL(trsv_bwd_step, dim3((unsigned)blocks), dim3(256), 0, s, nr, j, bq, L, ldl,
                                   Dinv + q * (int64_t)b * b, b, Y, (int64_t)kRhsGroup, Bc, ldb);
            }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t logdet(hipStream_t s, int64_t n, const double* L, int64_t ldl, double* out)
{
    hipLaunchKernelGGL(logdet_kernel, dim3(1), dim3(256), 0, s, n, L, ldl, out);
    return hipGetLastError();
}

}  // namespace gpc
