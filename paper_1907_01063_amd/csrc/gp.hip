// Gaussian-process pieces around the factor (section 1: the GP density is
// dominated by the covariance's Cholesky factor; section 4.2's GP regression)
// and the FP64 residual of iterative refinement:
//   kgen_se      K_ij = s2 exp(-1/2 sum_q (x_iq - x_jq)^2 / l_q^2) + sn2 [i == j]  (lower)
//   lbar         Lbar = tril(alpha z^T) - diag(1 / L_ii)
//   hypergrad_se dF/dtheta_q = scale * sum_{i>=j} Abar_ij dK_ij/dtheta_q,
//                theta = (s2, l_1..l_d, sn2)
//   value        f = -1/2 z^T z - 1/2 log|K|
//   symv         r = y - K x with K given by its lower triangle (FP64), and the
//                row sums of |K| (for the infinity norm)
// Every reduction runs in a fixed order (per-tile partial sums written to a
// workspace, then summed in tile order), so results do not depend on timing.
#include <algorithm>

#include "internal.hpp"

namespace gpc {
namespace {

constexpr int kT = 32;     // tile edge of the elementwise GP kernels
constexpr int kS = 64;     // tile edge of the SYMV

__device__ __forceinline__ double block_sum(double v, double* red)
{
    // fixed binary tree over 256 threads
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// One 32 x 32 tile per workgroup (256 threads, 4 elements each).
__global__ void __launch_bounds__(256)
kgen_se_kernel(int64_t n, int d, const double* X, const double* theta, double* K, int64_t ldk)
{
    __shared__ double xi[kT][kMaxGpDim], xj[kT][kMaxGpDim], il2[kMaxGpDim];
    const int64_t i0 = (int64_t)blockIdx.y * kT, j0 = (int64_t)blockIdx.x * kT;
    const int tid = threadIdx.x;
    if (j0 > i0 + kT - 1) {   // tile entirely above the diagonal
        for (int e = tid; e < kT * kT; e += 256) {
            const int64_t i = i0 + e / kT, j = j0 + e % kT;
            if (i < n && j < n) K[i * ldk + j] = 0.0;
        }
        return;
    }
    for (int e = tid; e < kT * d; e += 256) {
        const int r = e / d, q = e % d;
        xi[r][q] = i0 + r < n ? X[(i0 + r) * d + q] : 0.0;
        xj[r][q] = j0 + r < n ? X[(j0 + r) * d + q] : 0.0;
    }
    if (tid < d) il2[tid] = 1.0 / (theta[1 + tid] * theta[1 + tid]);
    __syncthreads();
    const double s2 = theta[0], sn2 = theta[d + 1];
    for (int e = tid; e < kT * kT; e += 256) {
        const int r = e / kT, c = e % kT;
        const int64_t i = i0 + r, j = j0 + c;
        if (i >= n || j >= n) continue;
        double v = 0.0;
        if (j <= i) {
            double r2 = 0.0;
            for (int q = 0; q < d; ++q) {
                const double df = xi[r][q] - xj[c][q];
                r2 += df * df * il2[q];
            }
            v = s2 * exp(-0.5 * r2);
            if (i == j) v += sn2;
        }
        K[i * ldk + j] = v;
    }
}

__global__ void lbar_kernel(int64_t n, const double* L, int64_t ldl, const double* alpha, const double* z,
                            double* Lbar, int64_t ldlb)
{
    const int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6);
    const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (i >= n || j >= n) return;
    double v = 0.0;
    if (j <= i) v = alpha[i] * z[j];
    if (j == i) v -= 1.0 / L[i * ldl + i];
    Lbar[i * ldlb + j] = v;
}

// Lower tiles only; tile t = (ti, tj), tj <= ti, in the usual triangular
// enumeration.  Each writes d+2 partial sums to part[t * (d+2) + q].
__global__ void __launch_bounds__(256)
hypergrad_tiles(int64_t n, int d, const double* X, const double* theta, const double* Ab, int64_t ldab,
                double* part)
{
    __shared__ double xi[kT][kMaxGpDim], xj[kT][kMaxGpDim], il2[kMaxGpDim], red[256];
    const int64_t t = blockIdx.x;
    int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > t) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    const int64_t tj = t - ti * (ti + 1) / 2;
    const int64_t i0 = ti * kT, j0 = tj * kT;
    const int tid = threadIdx.x;
    for (int e = tid; e < kT * d; e += 256) {
        const int r = e / d, q = e % d;
        xi[r][q] = i0 + r < n ? X[(i0 + r) * d + q] : 0.0;
        xj[r][q] = j0 + r < n ? X[(j0 + r) * d + q] : 0.0;
    }
    if (tid < d) il2[tid] = 1.0 / (theta[1 + tid] * theta[1 + tid]);
    __syncthreads();
    const double s2 = theta[0];
    // this thread's four elements of the tile, in a fixed order
    double av[4], ex[4];
    int rr[4], cc[4];
    bool diag[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = tid + 256 * k;
        rr[k] = e / kT;
        cc[k] = e % kT;
        const int64_t i = i0 + rr[k], j = j0 + cc[k];
        const bool ok = i < n && j <= i;
        av[k] = ok ? Ab[i * ldab + j] : 0.0;
        diag[k] = ok && i == j;
        double r2 = 0.0;
        for (int q = 0; q < d; ++q) {
            const double df = xi[rr[k]][q] - xj[cc[k]][q];
            r2 += df * df * il2[q];
        }
        ex[k] = ok ? exp(-0.5 * r2) : 0.0;
    }
    for (int q = 0; q < d + 2; ++q) {
        double sq = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (q == 0) {
                sq += av[k] * ex[k];
            } else if (q <= d) {
                const double df = xi[rr[k]][q - 1] - xj[cc[k]][q - 1];
                sq += av[k] * s2 * ex[k] * df * df * il2[q - 1] / theta[q];
            } else if (diag[k]) {
                sq += av[k];
            }
        }
        sq = block_sum(sq, red);
        if (tid == 0) part[t * (d + 2) + q] = sq;
    }
}

// grad[q] = scale * sum over tiles (tile order fixed by a per-thread stride
// and a fixed tree); one workgroup per component.
__global__ void __launch_bounds__(256)
reduce_parts(int64_t ntiles, int m, const double* part, const double* scale, double* grad)
{
    __shared__ double red[256];
    const int q = blockIdx.x;
    double s = 0.0;
#pragma unroll 8   // eight loads in flight; the additions keep their order
    for (int64_t t = threadIdx.x; t < ntiles; t += 256) s += part[t * m + q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) grad[q] = (scale ? *scale : 1.0) * s;
}

__global__ void __launch_bounds__(256)
gp_value_kernel(int64_t n, const double* a, const double* b, const double* logdet, double* f)
{
    __shared__ double red[256];
    double s = 0.0;
#pragma unroll 8   // eight loads in flight; the additions keep their order
    for (int64_t i = threadIdx.x; i < n; i += 256) s += a[i] * b[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *f = -0.5 * s - 0.5 * (*logdet);
}

// SYMV partials: workgroup per lower 64 x 64 block (bi, bj).  With the
// symmetric block S (lower-stored; the diagonal block mirrored),
// part[bi][bj] = S x[bj] and, off the diagonal, part[bj][bi] = S^T x[bi].
// absk: use |S|; x == nullptr: x is all ones.  part2 (if not null) also
// gets the same partials of |S| times a vector of ones (the row sums of |K|
// in the same pass over K).
__global__ void __launch_bounds__(256)
symv_blocks(int64_t n, const double* K, int64_t ldk, const double* x, int absk, double* part, double* part2,
            int64_t nb)
{
    __shared__ double S[kS][kS + 1];
    __shared__ double xr[kS], xc[kS], pr[4][kS], pc[4][kS];
    const int64_t t = blockIdx.x;
    int64_t bi = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > t) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int64_t bj = t - bi * (bi + 1) / 2;
    const int64_t i0 = bi * kS, j0 = bj * kS;
    const int tid = threadIdx.x;
    // lane c of wave w takes column c of rows w, w+4, ...: all 16 loads are
    // issued before the first is stored (the upper part of a diagonal block
    // is read from its mirror)
    {
        constexpr int R = kS * kS / 256;
        const int c = tid % kS, rw = tid / kS;
        const int64_t j = j0 + c;
        double v[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int64_t i = i0 + rw + 4 * k;
            const bool up = bi == bj && j > i;
            const int64_t off = up ? j * ldk + i : i * ldk + j;
            v[k] = (i < n && j < n) ? K[off] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) S[rw + 4 * k][c] = absk ? fabs(v[k]) : v[k];
    }
    if (tid < kS) {
        const int64_t j = j0 + tid, i = i0 + tid;
        xc[tid] = j < n ? (x ? x[j] : 1.0) : 0.0;
        xr[tid] = i < n ? (x ? x[i] : 1.0) : 0.0;
    }
    __syncthreads();
    const int row = tid & 63, part4 = tid >> 6;
    double a = 0.0, b = 0.0, a2 = 0.0, b2 = 0.0;
    for (int c = part4 * 16; c < part4 * 16 + 16; ++c) {
        a += S[row][c] * xc[c];   // (S x_c)[row]
        b += S[c][row] * xr[c];   // (S^T x_r)[row]
        if (part2) {              // entries outside K are zero in S
            a2 += fabs(S[row][c]);
            b2 += fabs(S[c][row]);
        }
    }
    pr[part4][row] = a;
    pc[part4][row] = b;
    __syncthreads();
    if (tid < kS) {
        part[(bi * nb + bj) * kS + tid] = ((pr[0][tid] + pr[1][tid]) + pr[2][tid]) + pr[3][tid];
        if (bi != bj) part[(bj * nb + bi) * kS + tid] = ((pc[0][tid] + pc[1][tid]) + pc[2][tid]) + pc[3][tid];
    }
    if (part2) {
        __syncthreads();
        pr[part4][row] = a2;
        pc[part4][row] = b2;
        __syncthreads();
        if (tid < kS) {
            part2[(bi * nb + bj) * kS + tid] = ((pr[0][tid] + pr[1][tid]) + pr[2][tid]) + pr[3][tid];
            if (bi != bj) part2[(bj * nb + bi) * kS + tid] = ((pc[0][tid] + pc[1][tid]) + pc[2][tid]) + pc[3][tid];
        }
    }
}

// out[i] = (y ? y[i] : 0) + sgn * sum_s part[i/64][s][i%64]: one workgroup
// per 64 rows, the nb partial sums of a row split into four consecutive
// ranges (s increasing within each, loads issued eight at a time) that are
// then added in range order.
__global__ void __launch_bounds__(256)
symv_finish(int64_t n, int64_t nb, const double* part, const double* y, double sgn, double* out)
{
    __shared__ double red[4][kS];
    const int r = threadIdx.x % kS, g = threadIdx.x / kS;
    const int64_t bi = blockIdx.x, i = bi * kS + r;
    const int64_t per = (nb + 3) / 4, t0 = g * per, t1 = min(nb, t0 + per);
    const double* p = part + (bi * nb) * kS + r;
    double s = 0.0;
    int64_t t = t0;
    for (; t + 8 <= t1; t += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = p[(t + k) * kS];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; t < t1; ++t) s += p[t * kS];
    red[g][r] = s;
    __syncthreads();
    if (g == 0 && i < n) out[i] = (y ? y[i] : 0.0) + sgn * (((red[0][r] + red[1][r]) + red[2][r]) + red[3][r]);
}

__global__ void __launch_bounds__(256)
eta_kernel(int64_t n, const double* r, const double* x, const double* y, const double* rowabs, double* eta)
{
    __shared__ double red[4][256];
    double mr = 0.0, mx = 0.0, my = 0.0, mk = 0.0;
#pragma unroll 8   // eight loads of each vector in flight
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        mr = fmax(mr, fabs(r[i]));
        mx = fmax(mx, fabs(x[i]));
        my = fmax(my, fabs(y[i]));
        mk = fmax(mk, rowabs[i]);
    }
    red[0][threadIdx.x] = mr;
    red[1][threadIdx.x] = mx;
    red[2][threadIdx.x] = my;
    red[3][threadIdx.x] = mk;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *eta = red[0][0] / (red[3][0] * red[1][0] + red[2][0]);
}

__global__ void axpy_kernel(int64_t n, const double* d, double* x)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] += d[i];
}

__global__ void copy_vec(int64_t n, const double* a, double* b)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void zero_vec(int64_t n, double* a)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

inline unsigned blocks256(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

}  // namespace

hipError_t gp_kgen_se(hipStream_t s, int64_t n, int d, const double* X, const double* theta, double* K, int64_t ldk)
{
    if (n <= 0) return hipSuccess;
    if (d < 1 || d > kMaxGpDim) return hipErrorInvalidValue;
    const unsigned t = (unsigned)((n + kT - 1) / kT);
    hipLaunchKernelGGL(kgen_se_kernel, dim3(t, t), dim3(256), 0, s, n, d, X, theta, K, ldk);
    return hipGetLastError();
}

hipError_t gp_lbar(hipStream_t s, int64_t n, const double* L, int64_t ldl, const double* alpha, const double* z,
                   double* Lbar, int64_t ldlb)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((n + 3) / 4));
    hipLaunchKernelGGL(lbar_kernel, grid, dim3(256), 0, s, n, L, ldl, alpha, z, Lbar, ldlb);
    return hipGetLastError();
}

int64_t gp_hypergrad_parts(int64_t n, int d)
{
    const int64_t t = (n + kT - 1) / kT;
    return std::max<int64_t>(1, t * (t + 1) / 2) * (d + 2);
}

hipError_t gp_hypergrad_se(hipStream_t s, int64_t n, int d, const double* X, const double* theta, const double* Ab,
                           int64_t ldab, const double* scale, double* grad, double* part)
{
    if (d < 1 || d > kMaxGpDim) return hipErrorInvalidValue;
    const int64_t t = (n + kT - 1) / kT;
    const int64_t ntiles = t * (t + 1) / 2;
    if (ntiles > 0)
        hipLaunchKernelGGL(hypergrad_tiles, dim3((unsigned)ntiles), dim3(256), 0, s, n, d, X, theta, Ab, ldab, part);
    hipLaunchKernelGGL(reduce_parts, dim3(d + 2), dim3(256), 0, s, ntiles, d + 2, part, scale, grad);
    return hipGetLastError();
}

hipError_t gp_value(hipStream_t s, int64_t n, const double* z, const double* logdet, double* f)
{
    hipLaunchKernelGGL(gp_value_kernel, dim3(1), dim3(256), 0, s, n, z, z, logdet, f);
    return hipGetLastError();
}

hipError_t gp_value_dot(hipStream_t s, int64_t n, const double* a, const double* b, const double* logdet, double* f)
{
    hipLaunchKernelGGL(gp_value_kernel, dim3(1), dim3(256), 0, s, n, a, b, logdet, f);
    return hipGetLastError();
}

int64_t symv_parts(int64_t n)
{
    const int64_t nb = (n + kS - 1) / kS;
    return std::max<int64_t>(1, nb * nb * kS);
}

hipError_t symv_lower(hipStream_t s, int64_t n, const double* K, int64_t ldk, const double* x, int absk,
                      const double* y, double sgn, double* out, double* part)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kS - 1) / kS;
    hipLaunchKernelGGL(symv_blocks, dim3((unsigned)(nb * (nb + 1) / 2)), dim3(256), 0, s, n, K, ldk, x, absk,
                       part, (double*)nullptr, nb);
    hipLaunchKernelGGL(symv_finish, dim3((unsigned)nb), dim3(256), 0, s, n, nb, part, y, sgn, out);
    return hipGetLastError();
}

hipError_t symv_lower_abs(hipStream_t s, int64_t n, const double* K, int64_t ldk, const double* x, const double* y,
                          double sgn, double* out, double* rowabs, double* part)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kS - 1) / kS;
    double* part2 = part + symv_parts(n);
    hipLaunchKernelGGL(symv_blocks, dim3((unsigned)(nb * (nb + 1) / 2)), dim3(256), 0, s, n, K, ldk, x, 0, part,
                       part2, nb);
    hipLaunchKernelGGL(symv_finish, dim3((unsigned)nb), dim3(256), 0, s, n, nb, part, y, sgn, out);
    hipLaunchKernelGGL(symv_finish, dim3((unsigned)nb), dim3(256), 0, s, n, nb, part2, (const double*)nullptr, 1.0,
                       rowabs);
    return hipGetLastError();
}

hipError_t refine_eta(hipStream_t s, int64_t n, const double* r, const double* x, const double* y,
                      const double* rowabs, double* eta)
{
    hipLaunchKernelGGL(eta_kernel, dim3(1), dim3(256), 0, s, n, r, x, y, rowabs, eta);
    return hipGetLastError();
}

hipError_t vec_axpy(hipStream_t s, int64_t n, const double* d, double* x)
{
    hipLaunchKernelGGL(axpy_kernel, dim3(blocks256(n)), dim3(256), 0, s, n, d, x);
    return hipGetLastError();
}

hipError_t vec_copy(hipStream_t s, int64_t n, const double* a, double* b)
{
    hipLaunchKernelGGL(copy_vec, dim3(blocks256(n)), dim3(256), 0, s, n, a, b);
    return hipGetLastError();
}

hipError_t vec_zero(hipStream_t s, int64_t n, double* a)
{
    hipLaunchKernelGGL(zero_vec, dim3(blocks256(n)), dim3(256), 0, s, n, a);
    return hipGetLastError();
}

}  // namespace gpc
