// Triangular solves with the factor and the log-determinant (the pieces a GP
// log-density needs: z = L^-1 y, alpha = L^-T z, log|K| = 2 sum log L_ii).
//
// The solves sweep the diagonal blocks of L (section 3.2 solves A x = b
// through the inverse of the triangle; here only the b x b diagonal blocks are
// inverted, and the off-diagonal blocks are applied as matrix-vector
// updates).  One launch per block step q, with lookahead: the step's small
// product z_q = D_q^-1 y_q (or D_q^-T y_q) was computed by the previous launch,
// so workgroup 0 of launch q applies z_q to the rows of the next block only and
// then forms z_{q+1} (double-buffered), while the other workgroups apply z_q to
// their share of the remaining rows.  The running right-hand side lives in a
// separate workspace; every reduction has a fixed order.
#include <algorithm>

#include "internal.hpp"

namespace gpc {
namespace {

constexpr int kRhsGroup = 8;   // right-hand sides handled per launch
constexpr int kRows = 64;      // rows per workgroup of the forward update

// Partial dot product of one quarter of a 128-wide row with z (thread quarter
// q covers columns q, q+4, ..., so the four threads of a row read adjacent
// words); all loads are independent and issued before any arithmetic.
__device__ __forceinline__ void quarter_dot(const double* row, int bq, int q, int nr,
                                            const double (*z)[kRhsGroup], double* acc)
{
    double v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const int c = q + 4 * k;
        v[k] = c < bq ? row[c] : 0.0;
    }
    for (int c = 0; c < nr; ++c) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const int cc = q + 4 * k;
            s += v[k] * (cc < bq ? z[cc][c] : 0.0);
        }
        acc[c] = s;
    }
}

// Combine the four quarter sums of each row (adjacent lanes), fixed order.
__device__ __forceinline__ double quad_sum(double v)
{
    const double a = __shfl_xor(v, 1, 64);      // partner in the pair
    const double p = (threadIdx.x & 1) ? a + v : v + a;
    const double b = __shfl_xor(p, 2, 64);
    return (threadIdx.x & 2) ? b + p : p + b;
}

// rows [r0, r1): Y[r] -= L[r, j:j+bq] z   (z in LDS, bq <= 128); four threads per row
__device__ void fwd_rows(int64_t r0, int64_t r1, int64_t j, int bq, int nr, const double* L, int64_t ldl,
                         const double (*z)[kRhsGroup], double* Y, int64_t ldy)
{
    const int q = threadIdx.x & 3;
    for (int64_t rb = r0; rb < r1; rb += 64) {
        const int64_t r = rb + (threadIdx.x >> 2);
        double acc[kRhsGroup];
        if (r < r1) quarter_dot(L + r * ldl + j, bq, q, nr, z, acc);
        else for (int c = 0; c < nr; ++c) acc[c] = 0.0;
        for (int c = 0; c < nr; ++c) {
            const double t = quad_sum(acc[c]);
            if (q == 0 && r < r1) Y[r * ldy + c] -= t;
        }
    }
}

// z_out = D^-1 y for the block rows [j, j+bq) of Y; writes z_out and B.
__device__ void fwd_diag(int64_t j, int bq, int nr, const double* Dq, int b, const double* Y, int64_t ldy,
                         double (*ys)[kRhsGroup], double* zout, double* B, int64_t ldb)
{
    for (int e = threadIdx.x; e < bq * nr; e += 256) ys[e / nr][e % nr] = Y[(j + e / nr) * ldy + e % nr];
    __syncthreads();
    const int q = threadIdx.x & 3;
    for (int i0 = 0; i0 < bq; i0 += 64) {
        const int i = i0 + (threadIdx.x >> 2);
        double acc[kRhsGroup];
        if (i < bq) quarter_dot(Dq + (int64_t)i * b, i + 1, q, nr, ys, acc);   // D^-1 is lower
        else for (int c = 0; c < nr; ++c) acc[c] = 0.0;
        for (int c = 0; c < nr; ++c) {
            const double t = quad_sum(acc[c]);
            if (q == 0 && i < bq) {
                zout[i * kRhsGroup + c] = t;
                B[(j + i) * ldb + c] = t;
            }
        }
    }
}

// Prologue of the forward sweep: z_0 from the first block.
__global__ void __launch_bounds__(256)
trsv_fwd_first(int nr, int bq, const double* D0, int b, const double* Y, int64_t ldy, double* zbuf, double* B,
               int64_t ldb)
{
    __shared__ double ys[kDiagMax][kRhsGroup];
    fwd_diag(0, bq, nr, D0, b, Y, ldy, ys, zbuf, B, ldb);
}

// Step q of the forward sweep (block rows [j, j+bq), next block [j+bq, j+bq+bq1)).
__global__ void __launch_bounds__(256)
trsv_fwd_step(int64_t n, int nr, int64_t j, int bq, int bq1, const double* L, int64_t ldl, const double* Dnext,
              int b, double* Y, int64_t ldy, const double* zcur, double* znext, double* B, int64_t ldb)
{
    __shared__ double z[kDiagMax][kRhsGroup];
    __shared__ double ys[kDiagMax][kRhsGroup];
    for (int e = threadIdx.x; e < bq * kRhsGroup; e += 256) z[e / kRhsGroup][e % kRhsGroup] = zcur[e];
    __syncthreads();
    const int64_t jn = j + bq;
    if (blockIdx.x == 0) {
        fwd_rows(jn, jn + bq1, j, bq, nr, L, ldl, z, Y, ldy);
        __syncthreads();
        fwd_diag(jn, bq1, nr, Dnext, b, Y, ldy, ys, znext, B, ldb);
    } else {
        const int64_t r0 = jn + bq1 + (int64_t)(blockIdx.x - 1) * kRows;
        fwd_rows(r0, min(n, r0 + kRows), j, bq, nr, L, ldl, z, Y, ldy);
    }
}

// acc[c] = sum_t L[j+t][r] z[t][c] over t in [t0, t1) for one column r
// (t1 - t0 <= 32); the loads are independent and issued together.
__device__ __forceinline__ void bwd_col(int64_t r, int64_t j, int t0, int t1, int nr, const double* L, int64_t ldl,
                                        const double (*z)[kRhsGroup], double* acc)
{
    double v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = t0 + k < t1 ? L[(j + t0 + k) * ldl + r] : 0.0;
    for (int c = 0; c < nr; ++c) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 32; ++k) s += v[k] * (t0 + k < t1 ? z[t0 + k][c] : 0.0);
        acc[c] = s;
    }
}

// cols [r0, r0+64): Y[r] -= sum_t L[j+t][r] z[t], t split over the 4 waves and
// combined in wave order.
__device__ void bwd_cols(int64_t r0, int64_t r1, int64_t j, int bq, int nr, const double* L, int64_t ldl,
                         const double (*z)[kRhsGroup], double* Y, int64_t ldy, double (*red)[64][kRhsGroup])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = r0 + lane;
    const int q4 = (bq + 3) / 4;
    const int t0 = min(bq, wave * q4), t1 = min(bq, t0 + q4);
    double acc[kRhsGroup];
    if (r < r1) bwd_col(r, j, t0, t1, nr, L, ldl, z, acc);
    else for (int c = 0; c < nr; ++c) acc[c] = 0.0;
    for (int c = 0; c < nr; ++c) red[wave][lane][c] = acc[c];
    __syncthreads();
    if (wave == 0 && r < r1)
        for (int c = 0; c < nr; ++c)
            Y[r * ldy + c] -= ((red[0][lane][c] + red[1][lane][c]) + red[2][lane][c]) + red[3][lane][c];
    __syncthreads();
}

// z_out = D^-T y for the block [j, j+bq) of Y; writes z_out and B.
__device__ void bwd_diag(int64_t j, int bq, int nr, const double* Dq, int b, const double* Y, int64_t ldy,
                         double (*ys)[kRhsGroup], double (*red)[64][kRhsGroup], double* zout, double* B,
                         int64_t ldb)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = threadIdx.x; e < bq * nr; e += 256) ys[e / nr][e % nr] = Y[(j + e / nr) * ldy + e % nr];
    __syncthreads();
    // z[i] = sum_{t >= i} D[t][i] y[t]: columns i over lanes (two halves), t over waves
    for (int h = 0; h < 2; ++h) {
        const int i = h * 64 + lane;
        const int q4 = (bq + 3) / 4;
        const int t0 = min(bq, wave * q4), t1 = min(bq, t0 + q4);
        double acc[kRhsGroup];
        for (int c = 0; c < nr; ++c) acc[c] = 0.0;
        if (i < bq) {
            double v[32];
#pragma unroll
            for (int k = 0; k < 32; ++k) {
                const int t = t0 + k;
                v[k] = (t < t1 && t >= i) ? Dq[(int64_t)t * b + i] : 0.0;   // D^-1 is lower
            }
            for (int c = 0; c < nr; ++c) {
                double sacc = 0.0;
#pragma unroll
                for (int k = 0; k < 32; ++k) sacc += v[k] * (t0 + k < t1 ? ys[t0 + k][c] : 0.0);
                acc[c] = sacc;
            }
        }
        for (int c = 0; c < nr; ++c) red[wave][lane][c] = acc[c];
        __syncthreads();
        if (wave == 0 && i < bq)
            for (int c = 0; c < nr; ++c) {
                const double p = ((red[0][lane][c] + red[1][lane][c]) + red[2][lane][c]) + red[3][lane][c];
                zout[i * kRhsGroup + c] = p;
                B[(j + i) * ldb + c] = p;
            }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256)
trsv_bwd_first(int nr, int64_t j, int bq, const double* Dq, int b, const double* Y, int64_t ldy, double* zbuf,
               double* B, int64_t ldb)
{
    __shared__ double ys[kDiagMax][kRhsGroup];
    __shared__ double red[4][64][kRhsGroup];
    bwd_diag(j, bq, nr, Dq, b, Y, ldy, ys, red, zbuf, B, ldb);
}

// Step q of the backward sweep: block [j, j+bq) solved (z_q in zcur); the
// previous block is [jp, j) with jp = j - bqp.
__global__ void __launch_bounds__(256)
trsv_bwd_step(int nr, int64_t j, int bq, int64_t jp, int bqp, const double* L, int64_t ldl, const double* Dprev,
              int b, double* Y, int64_t ldy, const double* zcur, double* znext, double* B, int64_t ldb)
{
    __shared__ double z[kDiagMax][kRhsGroup];
    __shared__ double ys[kDiagMax][kRhsGroup];
    __shared__ double red[4][64][kRhsGroup];
    for (int e = threadIdx.x; e < bq * kRhsGroup; e += 256) z[e / kRhsGroup][e % kRhsGroup] = zcur[e];
    __syncthreads();
    if (blockIdx.x == 0) {
        for (int64_t r0 = jp; r0 < j; r0 += 64) bwd_cols(r0, min(j, r0 + 64), j, bq, nr, L, ldl, z, Y, ldy, red);
        bwd_diag(jp, bqp, nr, Dprev, b, Y, ldy, ys, red, znext, B, ldb);
    } else {
        const int64_t r0 = (int64_t)(blockIdx.x - 1) * 64;
        if (r0 < jp) bwd_cols(r0, min(jp, r0 + 64), j, bq, nr, L, ldl, z, Y, ldy, red);
    }
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

int64_t trsm_workspace(int64_t n) { return (int64_t)kRhsGroup * n + 2 * kDiagMax * kRhsGroup; }

hipError_t trsm_blocked(hipStream_t s, int trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                        const double* Dinv, int b, double* B, int64_t ldb, double* Y)
{
    const int64_t nblk = (n + b - 1) / b;
    const int64_t bb = (int64_t)b * b;
    double* zb = Y + (int64_t)kRhsGroup * n;            // two z slots
    auto zslot = [&](int64_t q) { return zb + (q & 1) * kDiagMax * kRhsGroup; };
    for (int64_t c0 = 0; c0 < nrhs; c0 += kRhsGroup) {
        const int nr = (int)std::min<int64_t>(kRhsGroup, nrhs - c0);
        double* Bc = B + c0;
        hipLaunchKernelGGL(copy_cols, dim3((unsigned)((n * nr + 255) / 256)), dim3(256), 0, s, n, nr, Bc, ldb, Y,
                           (int64_t)kRhsGroup);
        if (!trans) {
            hipLaunchKernelGGL(trsv_fwd_first, dim3(1), dim3(256), 0, s, nr, (int)std::min<int64_t>(b, n), Dinv, b,
                               Y, (int64_t)kRhsGroup, zslot(0), Bc, ldb);
            for (int64_t q = 0; q + 1 < nblk; ++q) {
                const int64_t j = q * b;
                const int bq = b;
                const int bq1 = (int)std::min<int64_t>(b, n - j - b);
                const int64_t rest = n - (j + bq + bq1);
                const int64_t blocks = 1 + std::max<int64_t>(0, (rest + kRows - 1) / kRows);
                hipLaunchKernelGGL(trsv_fwd_step, dim3((unsigned)blocks), dim3(256), 0, s, n, nr, j, bq, bq1, L, ldl,
                                   Dinv + (q + 1) * bb, b, Y, (int64_t)kRhsGroup, zslot(q), zslot(q + 1), Bc, ldb);
            }
        } else {
            const int64_t jl = (nblk - 1) * b;
            hipLaunchKernelGGL(trsv_bwd_first, dim3(1), dim3(256), 0, s, nr, jl, (int)(n - jl), Dinv + (nblk - 1) * bb,
                               b, Y, (int64_t)kRhsGroup, zslot(nblk - 1), Bc, ldb);
            for (int64_t q = nblk - 1; q >= 1; --q) {
                const int64_t j = q * b, jp = j - b;
                const int bq = (int)std::min<int64_t>(b, n - j);
                const int64_t blocks = 1 + (jp + 63) / 64;
                hipLaunchKernelGGL(trsv_bwd_step, dim3((unsigned)blocks), dim3(256), 0, s, nr, j, bq, jp, b, L, ldl,
                                   Dinv + (q - 1) * bb, b, Y, (int64_t)kRhsGroup, zslot(q), zslot(q - 1), Bc, ldb);
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
