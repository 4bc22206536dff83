// Many covariance matrices of uneven order factored and differentiated in one
// persistent launch.
//
// Workgroups pull whole matrices from a device queue (an atomic counter over
// a task list sorted by decreasing order, so the largest start first) and run
// the blocked algorithms of section 3.3 on their matrix alone: the right-
// looking factor (diagonal block factor + inverse, panel product, lower-tile
// trailing update) and the blocked reverse sweep (panel solve, left and row
// updates, diagonal-block step), all with 64 x 64 MFMA tiles of the whole
// workgroup and the register-resident diagonal routines.  A matrix is touched
// by one workgroup only and every sum has a fixed order, so results do not
// depend on which workgroup takes which matrix.  Workgroups never wait for
// each other: each loops until the counter passes the end of the list.
#include <algorithm>

#include "diag.hpp"
#include "gemm_tile.hpp"

namespace gpc {
namespace {

constexpr int kBB = 64;                       // largest inner block of the batched path
typedef TileLds<double, 64, 64, 16> Lds64;

__device__ __forceinline__ GemmArgs ga(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                                       const double* B, int64_t ldb, double* C, int64_t ldc)
{
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda;
    g.B = B; g.ldb = ldb;
    g.C = C; g.ldc = ldc;
    g.kchunk = K > 0 ? K : 1;
    return g;
}

// All tiles of an M x N product, one after the other, by this workgroup.
// TI: MFMA type.  FP64 operands are converted on load when TI is float
// (the mixed form's FP32 products, FP32 accumulation, subtracted from FP64 C).
template <typename TI, bool AKM, bool BNK, int EPI, bool LOWER>
__device__ void wg_gemm(const GemmArgs& g, double* lds)
{
    static_assert(TileLds<TI, 64, 64, 16>::elems * sizeof(TI) <= Lds64::elems * sizeof(double), "tile LDS");
    if (g.M <= 0 || g.N <= 0) return;
    const int64_t tM = (g.M + 63) / 64, tN = (g.N + 63) / 64;
    const int64_t count = LOWER ? tM * (tM + 1) / 2 : tM * tN;
    for (int64_t t = 0; t < count; ++t) {
        int64_t tm, tn;
        if (LOWER) lower_tile(t, tm, tn);
        else { tm = t / tN; tn = t % tN; }
        gemm_tile<TI, 64, 64, 16, 2, 2, AKM, BNK, EPI, LOWER, double>(g, tm, tn, 0, (TI*)lds);
    }
    __syncthreads();   // results visible to the whole workgroup
}

__device__ void zero_upper_wg(int n, double* A, int64_t lda)
{
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += 256) {
        const int64_t r = e / n, c = e % n;
        if (c > r) A[r * lda + c] = 0.0;
    }
}

struct Scratch {
    double *X, *P, *W, *S, *T, *M;   // 64 x 64 each
};

template <typename TU>   // type of the trailing update's products (double, or float in the mixed form)
__device__ void factor_one(int n, int b, double* A, int32_t* info, const Scratch& w, double* lds,
                           double* colbuf, double* rowbuf, double* rls)
{
    const int64_t lda = n;
    for (int k = 0; k < n; k += b) {
        const int kb = min(b, n - k);
        diag_factor_inverse_g4<kBB / 16>(kb, A + k * lda + k, lda, w.X, kBB, info, k, colbuf, rowbuf, rls);
        __syncthreads();
        const int m = n - k - kb;
        if (m <= 0) continue;
        double* A21 = A + (int64_t)(k + kb) * lda + k;
        wg_gemm<double, false, true, EPI_STORE, false>(ga(m, kb, kb, A21, lda, w.X, kBB, A21, lda), lds);
        wg_gemm<TU, false, true, EPI_SUB, true>(ga(m, m, kb, A21, lda, A21, lda, A21 + kb, lda), lds);
    }
    zero_upper_wg(n, A, lda);
}

template <typename TU>   // type of the B-bar and R-bar products (double, or float in the mixed form)
__device__ void adjoint_one(int n, int b, const double* L, double* Lb, const Scratch& w, double* lds,
                            double* Ls, double* rowbuf)
{
    const int64_t ld = n;
    const int nblk = (n + b - 1) / b;
    for (int q = nblk - 1; q >= 0; --q) {
        const int j = q * b, k = min(n, j + b), bq = k - j, nr = n - k;
        const double* D = L + (int64_t)j * ld + j;
        double* Dbar = Lb + (int64_t)j * ld + j;
        double* Cbar = Lb + (int64_t)k * ld + j;
        diag_inverse<kBB / 16>(bq, D, ld, w.X, kBB, Ls, rowbuf);
        __syncthreads();
        if (nr > 0) {
            wg_gemm<double, false, false, EPI_STORE, false>(ga(nr, bq, bq, Cbar, ld, w.X, kBB, Cbar, ld), lds);
            if (j > 0)
                wg_gemm<TU, false, false, EPI_SUB, false>(
                    ga(nr, j, bq, Cbar, ld, L + (int64_t)j * ld, ld, Lb + (int64_t)k * ld, ld), lds);
            wg_gemm<double, true, false, EPI_STORE, false>(ga(bq, bq, nr, Cbar, ld, L + (int64_t)k * ld + j, ld, w.P, kBB),
                                                   lds);
        }
        // W = tril(Dbar - Cbar^T C)
        for (int base = 0; base < bq * bq; base += 16 * 256) {   // 16 loads per thread in flight
            double dv[16], pv[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int e = base + threadIdx.x + 256 * k;
                const int r = e / bq, c = e % bq;
                const bool in = e < bq * bq && r >= c;
                dv[k] = in ? Dbar[r * ld + c] : 0.0;
                pv[k] = in && nr > 0 ? w.P[r * kBB + c] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int e = base + threadIdx.x + 256 * k;
                const int r = e / bq, c = e % bq;
                if (e < bq * bq) w.W[r * kBB + c] = r >= c ? dv[k] - pv[k] : 0.0;
            }
        }
        __syncthreads();
        GemmArgs gp = ga(bq, bq, bq, D, ld, w.W, kBB, w.S, kBB);
        gp.a_lower = 1;
        wg_gemm<double, true, false, EPI_SYMLOW, false>(gp, lds);
        wg_gemm<double, false, false, EPI_STORE, false>(ga(bq, bq, bq, w.S, kBB, w.X, kBB, w.T, kBB), lds);
        GemmArgs gm = ga(bq, bq, bq, w.X, kBB, w.T, kBB, w.M, kBB);
        gm.C2 = Dbar;
        gm.ldc2 = ld;
        wg_gemm<double, true, false, EPI_PHI, false>(gm, lds);
        if (j > 0) {
            GemmArgs gr = ga(bq, j, bq + nr, Cbar, ld, L + (int64_t)j * ld, ld, Lb + (int64_t)j * ld, ld);
            gr.Ahead = w.M;
            gr.ldah = kBB;
            gr.head_k = bq;
            wg_gemm<TU, true, false, EPI_SUB, false>(gr, lds);
        }
    }
    zero_upper_wg(n, Lb, ld);
}

__global__ void __launch_bounds__(256)
batched_kernel(int nb, const BatchTask* tasks, double* Abase, double* Lbbase, int32_t* info, int32_t* counter,
               double* ws, int mode)
{
    __shared__ double lds[Lds64::elems];
    __shared__ double Ls[kBB * (kBB + 1)];
    __shared__ double colbuf[2 * 4 * kBB], rowbuf[2 * 4 * kBB], rls[kBB];
    __shared__ int s_task;
    double* mine = ws + (int64_t)blockIdx.x * 6 * kBB * kBB;
    const Scratch w{mine, mine + kBB * kBB, mine + 2 * kBB * kBB, mine + 3 * kBB * kBB, mine + 4 * kBB * kBB,
                    mine + 5 * kBB * kBB};
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_task = atomicAdd(counter, 1);
        __syncthreads();
        const int t = s_task;
        if (t >= nb) break;
        const BatchTask T = tasks[t];
        if (mode & 1) {
            if (threadIdx.x == 0) info[T.idx] = 0;
            __syncthreads();
            if (mode & 4) factor_one<float>(T.n, T.block, Abase + T.off, info + T.idx, w, lds, colbuf, rowbuf, rls);
            else factor_one<double>(T.n, T.block, Abase + T.off, info + T.idx, w, lds, colbuf, rowbuf, rls);
            __syncthreads();
        }
        if (mode & 2) {
            if (mode & 4) adjoint_one<float>(T.n, T.block, Abase + T.off, Lbbase + T.off, w, lds, Ls, rowbuf);
            else adjoint_one<double>(T.n, T.block, Abase + T.off, Lbbase + T.off, w, lds, Ls, rowbuf);
        }
    }
}

// Synthetic SPD matrix for the tuner: A_ij = 1 / (1 + |i - j|) off the
// diagonal, A_ii = n (strictly diagonally dominant); Lbar_ij = 1 / (1 + i + j).
__global__ void spd_fill_kernel(int64_t n, double* A, double* Lb)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * n) return;
    const int64_t i = e / n, j = e % n;
    A[e] = i == j ? (double)n : 1.0 / (1.0 + (double)(i > j ? i - j : j - i));
    Lb[e] = j <= i ? 1.0 / (1.0 + (double)(i + j)) : 0.0;
}

}  // namespace

hipError_t spd_test_fill(hipStream_t s, int64_t n, double* A, double* Lb, int64_t off)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(spd_fill_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, n, A + off,
                       Lb + off);
    return hipGetLastError();
}

int64_t batched_scratch_doubles(int wgs) { return (int64_t)wgs * 6 * kBB * kBB; }

int batched_max_block() { return kBB; }

hipError_t batched_launch(hipStream_t s, int nb, const BatchTask* tasks, double* Abase, double* Lbbase,
                          int32_t* info, int32_t* counter, double* ws, int wgs, int mode)
{
    hipError_t e = fill_i32(s, counter, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batched_kernel, dim3((unsigned)wgs), dim3(256), 0, s, nb, tasks, Abase, Lbbase, info,
                       counter, ws, mode);
    return hipGetLastError();
}

}  // namespace gpc
