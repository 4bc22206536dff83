// Triangular solves with the factor and the log-determinant (the pieces a GP
// log-density needs: z = L^-1 y, alpha = L^-T z, log|K| = 2 sum log L_ii).
//
// The solves sweep the b x b diagonal blocks of L (section 3.2 solves A x = b
// through the inverse of the triangle; here only the diagonal blocks are
// inverted, and the off-diagonal blocks are applied as matrix-vector
// updates).  One launch per block step q, with lookahead: with the coupling
// blocks Cf_{q+1} = Dinv_{q+1} L_{q+1,q} formed beforehand, the next block's
// solution is z_{q+1} = Dinv_{q+1} y_{q+1} - Cf_{q+1} z_q, where y_{q+1}
// already holds the updates of all earlier blocks.  So in launch q a few
// workgroups each form 16 rows of z_{q+1} directly from z_q, with no wait on
// anything else in the launch, while the other workgroups apply z_q to the
// rows below block q+1.  The transposed sweep is the mirror image with
// Cb_q = L_{q+1,q} Dinv_q (x_{q-1} = Dinv_{q-1}^T y_{q-1} - Cb_{q-1}^T x_q).
// The running right-hand side lives in a separate workspace; every
// reduction has a fixed order.
#include <algorithm>

#include "internal.hpp"

namespace gpc {
namespace {

constexpr int kRhsGroup = 8;   // right-hand sides handled per launch
constexpr int kSolveMax = 256; // largest block size of the sweeps

constexpr int kRows = 64;      // rows per workgroup of the forward update

// NRC: 1 for one right-hand side (the lookahead's operand rows are then
// loaded before the wait for y and z), kRhsGroup otherwise.

// rows [r0, r1): Y[r] -= L[r, j:j+BS] z (z in LDS).  TPR = BS/32 threads per
// row, thread slot q covering columns q, q+TPR, ... (adjacent threads read
// adjacent words); all loads issued before any arithmetic; the TPR partial
// sums of a row are combined in a fixed order.
template <int BS>
__device__ void fwd_rows(int64_t r0, int64_t r1, int64_t j, int nr, const double* L, int64_t ldl,
                         const double (*z)[kRhsGroup], double* Y, int64_t ldy)
{
    constexpr int TPR = BS / 32, RPP = 256 / TPR;   // rows per pass
    const int q = threadIdx.x % TPR;
    for (int64_t rb = r0; rb < r1; rb += RPP) {
        const int64_t r = rb + threadIdx.x / TPR;
        double acc[kRhsGroup];
#pragma unroll
        for (int c = 0; c < kRhsGroup; ++c) acc[c] = 0.0;
        if (r < r1) {
            const double* row = L + r * ldl + j;
            double v[32];
#pragma unroll
            for (int k = 0; k < 32; ++k) v[k] = row[q + TPR * k];
            for (int c = 0; c < nr; ++c) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < 32; ++k) t += v[k] * z[q + TPR * k][c];
                acc[c] = t;
            }
        }
        for (int c = 0; c < nr; ++c) {
            double v = acc[c];
#pragma unroll
            for (int w = 1; w < TPR; w <<= 1) {
                const double o = __shfl_xor(v, w, 64);
                v = (threadIdx.x & w) ? o + v : v + o;
            }
            if (q == 0 && r < r1) Y[r * ldy + c] -= v;
        }
    }
}

// cols [r0, r1) (at most 64): Y[r] -= sum_t L[j+t][r] z[t] over t < bq, t
// split over the 4 waves (BS/4 each) and combined in wave order.
template <int BS>
__device__ void bwd_cols(int64_t r0, int64_t r1, int64_t j, int bq, int nr, const double* L, int64_t ldl,
                         const double (*z)[kRhsGroup], double* Y, int64_t ldy, double (*red)[64][kRhsGroup])
{
    constexpr int TW = BS / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = r0 + lane;
    const int t0 = wave * TW;
    double acc[kRhsGroup];
#pragma unroll
    for (int c = 0; c < kRhsGroup; ++c) acc[c] = 0.0;
    if (r < r1) {
        double v[TW];
#pragma unroll
        for (int k = 0; k < TW; ++k) v[k] = t0 + k < bq ? L[(j + t0 + k) * ldl + r] : 0.0;
#pragma unroll
        for (int c = 0; c < kRhsGroup; ++c) {
            if (c < nr) {
                double sacc = 0.0;
#pragma unroll
                for (int k = 0; k < TW; ++k) sacc += v[k] * z[t0 + k][c];
                acc[c] = sacc;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kRhsGroup; ++c)
        if (c < nr) red[wave][lane][c] = acc[c];
    __syncthreads();
    if (wave == 0 && r < r1)
        for (int c = 0; c < nr; ++c)
            Y[r * ldy + c] -= ((red[0][lane][c] + red[1][lane][c]) + red[2][lane][c]) + red[3][lane][c];
    __syncthreads();
}

// Forward lookahead: rows [i0, i0+16) of z_next = Dinv y_next - Cf z_cur for
// the block [jn, jn + bn) (bn <= BS rows; z_cur has bc entries, 0 if none).
// 16 threads per row, thread slot s covers columns s, s+16, ...; the 16
// partial sums of a row are combined in a fixed order.
template <int BS>
__device__ void fwd_look(int i0, int bn, int bc, int nr, const double* Dn, const double* Cf,
                         const double* Y, int64_t jn, int64_t ldy, const double* zcur, double* znext, double* B,
                         int64_t ldb)
{
    __shared__ double ys[BS][kRhsGroup];
    __shared__ double zs[BS][kRhsGroup];
    for (int e = threadIdx.x; e < BS * kRhsGroup; e += 256) {
        const int r = e / kRhsGroup, c = e % kRhsGroup;
        ys[r][c] = (r < bn && c < nr) ? Y[(jn + r) * ldy + c] : 0.0;
        zs[r][c] = (r < bc && c < nr) ? zcur[e] : 0.0;
    }
    __syncthreads();
    const int sl = threadIdx.x & 15;
    const int i = i0 + (threadIdx.x >> 4);
    double acc[kRhsGroup];
#pragma unroll
    for (int c = 0; c < kRhsGroup; ++c) acc[c] = 0.0;
    if (i < bn) {
        double dv[BS / 16], cv[BS / 16];
#pragma unroll
        for (int m = 0; m < BS / 16; ++m) {
            const int k = sl + 16 * m;
            dv[m] = k <= i ? Dn[(int64_t)i * BS + k] : 0.0;            // Dinv is lower
            cv[m] = (Cf && k < bc) ? Cf[(int64_t)i * BS + k] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < kRhsGroup; ++c) {
            double t = 0.0;
#pragma unroll
            for (int m = 0; m < BS / 16; ++m) t += dv[m] * ys[sl + 16 * m][c] - cv[m] * zs[sl + 16 * m][c];
            acc[c] = t;
        }
    }
#pragma unroll
    for (int c = 0; c < kRhsGroup; ++c) {
        double v = acc[c];
#pragma unroll
        for (int w = 1; w < 16; w <<= 1) {
            const double o = __shfl_xor(v, w, 64);
            v = (sl & w) ? o + v : v + o;
        }
        acc[c] = v;
    }
    if (sl == 0 && i < bn)
        for (int c = 0; c < nr; ++c) {
            znext[i * kRhsGroup + c] = acc[c];
            B[(jn + i) * ldb + c] = acc[c];
        }
}

// Forward lookahead, one right-hand side: rows [i0, i0+16) of
// z_next = Dinv y_next - Cf z_cur for the block [jn, jn + bn) (bn <= BS rows;
// z_cur has bc entries, 0 if none).
// 16 threads per row, thread slot s covers columns s, s+16, ...; the rows of
// Dinv and Cf are loaded before y and z; the 16 partial sums of a row are
// combined in a fixed order.
template <int BS>
__device__ void fwd_look1(int i0, int bn, int bc, int nr, const double* Dn, const double* Cf,
                         const double* Y, int64_t jn, int64_t ldy, const double* zcur, double* znext, double* B,
                         int64_t ldb)
{
    __shared__ double ys[BS][1];
    __shared__ double zs[BS][1];
    const int sl = threadIdx.x & 15;
    const int i = i0 + (threadIdx.x >> 4);
    double dv[BS / 16], cv[BS / 16];
#pragma unroll
    for (int m = 0; m < BS / 16; ++m) {
        const int k = sl + 16 * m;
        dv[m] = (i < bn && k <= i) ? Dn[(int64_t)i * BS + k] : 0.0;            // Dinv is lower
        cv[m] = (i < bn && Cf && k < bc) ? Cf[(int64_t)i * BS + k] : 0.0;
    }
    for (int e = threadIdx.x; e < BS * 1; e += 256) {
        const int r = e / 1, c = e % 1;
        ys[r][c] = (r < bn && c < nr) ? Y[(jn + r) * ldy + c] : 0.0;
        zs[r][c] = (r < bc && c < nr) ? zcur[r * kRhsGroup + c] : 0.0;
    }
    __syncthreads();
    double t[1];
#pragma unroll
    for (int c = 0; c < 1; ++c) {
        t[c] = 0.0;
#pragma unroll
        for (int m = 0; m < BS / 16; ++m) t[c] += dv[m] * ys[sl + 16 * m][c] - cv[m] * zs[sl + 16 * m][c];
    }
#pragma unroll
    for (int c = 0; c < 1; ++c) {
#pragma unroll
        for (int w = 1; w < 16; w <<= 1) {
            const double o = __shfl_xor(t[c], w, 64);
            t[c] = (sl & w) ? o + t[c] : t[c] + o;
        }
        if (sl == 0 && i < bn && c < nr) {
            znext[i * kRhsGroup + c] = t[c];
            B[(jn + i) * ldb + c] = t[c];
        }
    }
}

// Backward lookahead: rows [i0, i0+16) of x_prev = Dinv^T y_prev - Cb^T x_cur
// for the block [jp, jp + bp) (x_cur has bc entries, 0 if none).  Thread
// (t-slot g, row i0 + l) covers t = g, g+16, ...; partial sums over the 16
// t-slots are combined in a fixed order through LDS.
template <int BS>
__device__ void bwd_look(int i0, int bp, int bc, int nr, const double* Dp, const double* Cb,
                         const double* Y, int64_t jp, int64_t ldy, const double* xcur, double* xnext, double* B,
                         int64_t ldb)
{
    __shared__ double ys[BS][kRhsGroup];
    __shared__ double xs[BS][kRhsGroup];
    __shared__ double red[16][16][kRhsGroup];
    for (int e = threadIdx.x; e < BS * kRhsGroup; e += 256) {
        const int r = e / kRhsGroup, c = e % kRhsGroup;
        ys[r][c] = (r < bp && c < nr) ? Y[(jp + r) * ldy + c] : 0.0;
        xs[r][c] = (r < bc && c < nr) ? xcur[e] : 0.0;
    }
    __syncthreads();
    const int l = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int i = i0 + l;
    double acc[kRhsGroup];
#pragma unroll
    for (int c = 0; c < kRhsGroup; ++c) acc[c] = 0.0;
    if (i < bp) {
        double dv[BS / 16], cv[BS / 16];
#pragma unroll
        for (int m = 0; m < BS / 16; ++m) {
            const int t = g + 16 * m;
            dv[m] = (t >= i && t < bp) ? Dp[(int64_t)t * BS + i] : 0.0;   // (Dinv^T)[i][t], Dinv lower
            cv[m] = (Cb && t < bc) ? Cb[(int64_t)t * BS + i] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < kRhsGroup; ++c) {
            double t2 = 0.0;
#pragma unroll
            for (int m = 0; m < BS / 16; ++m) t2 += dv[m] * ys[g + 16 * m][c] - cv[m] * xs[g + 16 * m][c];
            acc[c] = t2;
        }
    }
#pragma unroll
    for (int c = 0; c < kRhsGroup; ++c) red[g][l][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < 16 && i0 + (int)threadIdx.x < bp) {
        const int ii = i0 + threadIdx.x;
        for (int c = 0; c < nr; ++c) {
            double v = 0.0;
            for (int gg = 0; gg < 16; ++gg) v += red[gg][threadIdx.x][c];
            xnext[ii * kRhsGroup + c] = v;
            B[(jp + ii) * ldb + c] = v;
        }
    }
}

// Backward lookahead, one right-hand side: rows [i0, i0+16) of
// x_prev = Dinv^T y_prev - Cb^T x_cur for the block [jp, jp + bp) (x_cur has
// bc entries, 0 if none).  Thread
// (t-slot g, row i0 + l) covers t = g, g+16, ...; the columns of Dinv and Cb
// are loaded before y and x; partial sums over the 16 t-slots are combined in
// a fixed order through LDS.
template <int BS>
__device__ void bwd_look1(int i0, int bp, int bc, int nr, const double* Dp, const double* Cb,
                         const double* Y, int64_t jp, int64_t ldy, const double* xcur, double* xnext, double* B,
                         int64_t ldb)
{
    __shared__ double ys[BS][1];
    __shared__ double xs[BS][1];
    __shared__ double red[16][16][1];
    const int l = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int i = i0 + l;
    double dv[BS / 16], cv[BS / 16];
#pragma unroll
    for (int m = 0; m < BS / 16; ++m) {
        const int t = g + 16 * m;
        dv[m] = (i < bp && t >= i && t < bp) ? Dp[(int64_t)t * BS + i] : 0.0;   // (Dinv^T)[i][t], Dinv lower
        cv[m] = (i < bp && Cb && t < bc) ? Cb[(int64_t)t * BS + i] : 0.0;
    }
    for (int e = threadIdx.x; e < BS * 1; e += 256) {
        const int r = e / 1, c = e % 1;
        ys[r][c] = (r < bp && c < nr) ? Y[(jp + r) * ldy + c] : 0.0;
        xs[r][c] = (r < bc && c < nr) ? xcur[r * kRhsGroup + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 1; ++c) {
        double t2 = 0.0;
#pragma unroll
        for (int m = 0; m < BS / 16; ++m) t2 += dv[m] * ys[g + 16 * m][c] - cv[m] * xs[g + 16 * m][c];
        red[g][l][c] = t2;
    }
    __syncthreads();
    if (threadIdx.x < 16 && i0 + (int)threadIdx.x < bp) {
        const int ii = i0 + threadIdx.x;
        for (int c = 0; c < nr; ++c) {
            double v = 0.0;
            for (int gg = 0; gg < 16; ++gg) v += red[gg][threadIdx.x][c];
            xnext[ii * kRhsGroup + c] = v;
            B[(jp + ii) * ldb + c] = v;
        }
    }
}

// Forward sweep, launch q (q = -1: z_0 only).  Workgroups < BS/16 form the
// next block's z; the rest update the rows below the next block with z_q.
template <int BS, int NRC>
__global__ void __launch_bounds__(256)
trsv_fwd(int64_t n, int nr, int64_t q, const double* L, int64_t ldl, const double* Dinv, const double* Cf,
         double* Y, int64_t ldy, const double* zcur, double* znext, double* B, int64_t ldb)
{
    constexpr int kLook = BS / 16;
    const int64_t jn = (q + 1) * BS;                      // next block
    const int bn = (int)min((int64_t)BS, n - jn);
    const int bc = q >= 0 ? BS : 0;                       // block q is full whenever a next block exists
    if (blockIdx.x < kLook) {
        if constexpr (NRC == 1)
            fwd_look1<BS>(blockIdx.x * 16, bn, bc, nr, Dinv + (q + 1) * BS * BS,
                          q >= 0 ? Cf + (q + 1) * BS * BS : nullptr, Y, jn, ldy, zcur, znext, B, ldb);
        else
            fwd_look<BS>(blockIdx.x * 16, bn, bc, nr, Dinv + (q + 1) * BS * BS,
                         q >= 0 ? Cf + (q + 1) * BS * BS : nullptr, Y, jn, ldy, zcur, znext, B, ldb);
    } else {
        __shared__ double z[BS][kRhsGroup];
        for (int e = threadIdx.x; e < BS * kRhsGroup; e += 256) z[e / kRhsGroup][e % kRhsGroup] = zcur[e];
        __syncthreads();
        const int64_t r0 = jn + bn + (int64_t)(blockIdx.x - kLook) * kRows;
        fwd_rows<BS>(r0, min(n, r0 + kRows), q * BS, nr, L, ldl, z, Y, ldy);
    }
}

// Backward sweep, launch q (q = nblk: x_{nblk-1} only): workgroups < BS/16
// form x_{q-1}; the rest update the columns left of block q-1 with x_q.
template <int BS, int NRC>
__global__ void __launch_bounds__(256)
trsv_bwd(int64_t n, int nr, int64_t q, int64_t nblk, const double* L, int64_t ldl, const double* Dinv,
         const double* Cb, double* Y, int64_t ldy, const double* xcur, double* xnext, double* B, int64_t ldb)
{
    constexpr int kLook = BS / 16;
    const int64_t jp = (q - 1) * BS;                      // previous block
    const int bp = (int)min((int64_t)BS, n - jp);
    const int bc = q < nblk ? (int)min((int64_t)BS, n - q * BS) : 0;
    if (blockIdx.x < kLook) {
        if constexpr (NRC == 1)
            bwd_look1<BS>(blockIdx.x * 16, bp, bc, nr, Dinv + (q - 1) * BS * BS,
                          q < nblk ? Cb + (q - 1) * BS * BS : nullptr, Y, jp, ldy, xcur, xnext, B, ldb);
        else
            bwd_look<BS>(blockIdx.x * 16, bp, bc, nr, Dinv + (q - 1) * BS * BS,
                         q < nblk ? Cb + (q - 1) * BS * BS : nullptr, Y, jp, ldy, xcur, xnext, B, ldb);
    } else {
        __shared__ double z[BS][kRhsGroup];
        __shared__ double red[4][64][kRhsGroup];
        for (int e = threadIdx.x; e < BS * kRhsGroup; e += 256) z[e / kRhsGroup][e % kRhsGroup] = xcur[e];
        __syncthreads();
        const int64_t r0 = (int64_t)(blockIdx.x - kLook) * 64;
        if (r0 < jp) bwd_cols<BS>(r0, min(jp, r0 + 64), q * BS, bc, nr, L, ldl, z, Y, ldy, red);
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

int64_t trsm_workspace(int64_t n) { return (int64_t)kRhsGroup * n + 2 * kSolveMax * kRhsGroup; }

hipError_t trsm_couplings(hipStream_t s, int trans, int64_t n, const double* L, int64_t ldl, const double* Dinv,
                          int b, double* C)
{
    const int64_t nblk = (n + b - 1) / b;
    if (nblk < 2) return hipSuccess;
    const int64_t bb = (int64_t)b * b;
    const int64_t last = nblk - 1;
    const int bl = (int)(n - last * b);                   // rows of the last block
    if (!trans) {
        // Cf_q = Dinv_q L_{q,q-1}, q = 1 .. nblk-1 (the last one with bl rows)
        const int64_t full = bl == b ? last : last - 1;   // full blocks among q = 1 .. last
        if (full >= 1) {
            GemmArgs g{};
            g.M = b; g.N = b; g.K = b;
            g.A = Dinv + bb; g.lda = b; g.a_lower = 1;
            g.B = L + (int64_t)b * ldl; g.ldb = ldl;
            g.C = C + bb; g.ldc = b;
            g.kchunk = b;
            g.bsA = bb; g.bsB = (int64_t)b * ldl + b; g.bsC = bb;
            hipError_t e = gemm_f64(s, TILE_128, false, false, EPI_STORE, false, g, 1, (int)full);
            if (e != hipSuccess) return e;
        }
        if (bl != b) {
            GemmArgs g{};
            g.M = bl; g.N = b; g.K = bl;
            g.A = Dinv + last * bb; g.lda = b; g.a_lower = 1;
            g.B = L + last * b * ldl + (last - 1) * b; g.ldb = ldl;
            g.C = C + last * bb; g.ldc = b;
            g.kchunk = bl;
            hipError_t e = gemm_f64(s, TILE_128, false, false, EPI_STORE, false, g, 1, 1);
            if (e != hipSuccess) return e;
        }
    } else {
        // Cb_q = L_{q+1,q} Dinv_q, q = 0 .. nblk-2 (rows of block q+1)
        const int64_t full = bl == b ? last : last - 1;   // q with a full block q+1
        if (full >= 1) {
            GemmArgs g{};
            g.M = b; g.N = b; g.K = b;
            g.A = L + (int64_t)b * ldl; g.lda = ldl;
            g.B = Dinv; g.ldb = b;
            g.C = C; g.ldc = b;
            g.kchunk = b;
            g.bsA = (int64_t)b * ldl + b; g.bsB = bb; g.bsC = bb;
            hipError_t e = gemm_f64(s, TILE_128, false, false, EPI_STORE, false, g, 1, (int)full);
            if (e != hipSuccess) return e;
        }
        if (bl != b) {
            const int64_t q = last - 1;
            GemmArgs g{};
            g.M = bl; g.N = b; g.K = b;
            g.A = L + last * b * ldl + q * b; g.lda = ldl;
            g.B = Dinv + q * bb; g.ldb = b;
            g.C = C + q * bb; g.ldc = b;
            g.kchunk = b;
            hipError_t e = gemm_f64(s, TILE_128, false, false, EPI_STORE, false, g, 1, 1);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

namespace {
template <int BS>
hipError_t sweep(hipStream_t s, int trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                 const double* Dinv, const double* Cpl, double* B, int64_t ldb, double* Y)
{
    constexpr int kLook = BS / 16;
    const int64_t nblk = (n + BS - 1) / BS;
    double* zb = Y + (int64_t)kRhsGroup * n;            // two z slots
    auto zslot = [&](int64_t q) { return zb + (q & 1) * kSolveMax * kRhsGroup; };
    for (int64_t c0 = 0; c0 < nrhs; c0 += kRhsGroup) {
        const int nr = (int)std::min<int64_t>(kRhsGroup, nrhs - c0);
        double* Bc = B + c0;
        hipLaunchKernelGGL(copy_cols, dim3((unsigned)((n * nr + 255) / 256)), dim3(256), 0, s, n, nr, Bc, ldb, Y,
                           (int64_t)kRhsGroup);
        if (!trans) {
            for (int64_t q = -1; q + 1 < nblk; ++q) {
                const int64_t jn = (q + 1) * BS;
                const int64_t rest = n - std::min(n, jn + BS);
                const int64_t blocks = kLook + (q >= 0 ? (rest + kRows - 1) / kRows : 0);
                if (nr == 1)
                    hipLaunchKernelGGL((trsv_fwd<BS, 1>), dim3((unsigned)blocks), dim3(256), 0, s, n, nr, q, L, ldl,
                                       Dinv, Cpl, Y, (int64_t)kRhsGroup, zslot(q), zslot(q + 1), Bc, ldb);
                else
                    hipLaunchKernelGGL((trsv_fwd<BS, kRhsGroup>), dim3((unsigned)blocks), dim3(256), 0, s, n, nr, q,
                                       L, ldl, Dinv, Cpl, Y, (int64_t)kRhsGroup, zslot(q), zslot(q + 1), Bc, ldb);
            }
        } else {
            for (int64_t q = nblk; q >= 1; --q) {
                const int64_t jp = (q - 1) * BS;
                const int64_t blocks = kLook + (q < nblk ? (jp + 63) / 64 : 0);
                if (nr == 1)
                    hipLaunchKernelGGL((trsv_bwd<BS, 1>), dim3((unsigned)blocks), dim3(256), 0, s, n, nr, q, nblk, L,
                                       ldl, Dinv, Cpl, Y, (int64_t)kRhsGroup, zslot(q), zslot(q - 1), Bc, ldb);
                else
                    hipLaunchKernelGGL((trsv_bwd<BS, kRhsGroup>), dim3((unsigned)blocks), dim3(256), 0, s, n, nr, q,
                                       nblk, L, ldl, Dinv, Cpl, Y, (int64_t)kRhsGroup, zslot(q), zslot(q - 1), Bc, ldb);
            }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

hipError_t trsm_blocked(hipStream_t s, int trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                        const double* Dinv, const double* Cpl, int b, double* B, int64_t ldb, double* Y)
{
    if (b == 128) return sweep<128>(s, trans, n, nrhs, L, ldl, Dinv, Cpl, B, ldb, Y);
    if (b == 256) return sweep<256>(s, trans, n, nrhs, L, ldl, Dinv, Cpl, B, ldb, Y);
    return hipErrorInvalidValue;
}

hipError_t logdet(hipStream_t s, int64_t n, const double* L, int64_t ldl, double* out)
{
    hipLaunchKernelGGL(logdet_kernel, dim3(1), dim3(256), 0, s, n, L, ldl, out);
    return hipGetLastError();
}

}  // namespace gpc
