// MFMA tile body shared by the stand-alone GEMM kernels and the persistent
// batched kernel.  See gemm.hip for the scheme.
#pragma once

#include "internal.hpp"

namespace gpc {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4v acc_t;
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lr, int r) { return lr + 4 * r; }
};
template <> struct Mfma<float> {
    typedef f4v acc_t;
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lr, int r) { return 4 * lr + r; }
};

// Tile (ti, tj), tj <= ti, of index b in the row-by-row enumeration of the
// lower triangle of tiles.
__device__ __forceinline__ void lower_tile(int64_t b, int64_t& ti, int64_t& tj)
{
    int64_t t = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (t * (t + 1) / 2 > b) --t;
    while ((t + 1) * (t + 2) / 2 <= b) ++t;
    ti = t;
    tj = b - t * (t + 1) / 2;
}

template <typename TI, int BM, int BN, int BK>
struct TileLds {
    static constexpr int PAD = sizeof(TI) == 8 ? 2 : 4;
    static constexpr int elems = 2 * BK * (BM + PAD) + 2 * BK * (BN + PAD);
};

// One BM x BN output tile (tile row tm, tile column tn, split slice z) computed
// by the whole workgroup (WM x WN waves).  lds: TileLds<...>::elems elements.
// Ends with all LDS reads done, so calls may follow each other directly.
template <typename TI, int BM, int BN, int BK, int WM, int WN, bool AKM, bool BNK, int EPI, bool LOWER>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int64_t tm, int64_t tn, int64_t z, TI* lds)
{
    constexpr int NT = WM * WN * 64;
    constexpr int WTM = BM / WM, WTN = BN / WN;  // wave sub-tile
    constexpr int FM = WTM / 16, FN = WTN / 16;  // MFMA blocks per wave
    constexpr int PAD = TileLds<TI, BM, BN, BK>::PAD;
    constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
    // per-load step of the strided index: rows (MK/NK) or k rows (KM/KN)
    constexpr int ASTEP = AKM ? NT / BM : NT / BK;
    constexpr int BSTEP = BNK ? NT / BK : NT / BN;
    static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile/thread mismatch");
    typedef typename Mfma<TI>::acc_t acc_t;

    typedef TI RowA[BM + PAD];
    typedef TI RowB[BN + PAD];
    RowA* sA0 = (RowA*)lds;
    RowB* sB0 = (RowB*)(lds + 2 * BK * (BM + PAD));
    auto sA = [&](int buf, int kk) -> RowA& { return sA0[buf * BK + kk]; };
    auto sB = [&](int buf, int kk) -> RowB& { return sB0[buf * BK + kk]; };

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int64_t kbeg = z * g.kchunk;
    const int64_t kend = min(g.K, kbeg + g.kchunk);

    // no __restrict__: the in-place panel products write the rows they read
    const TI* Ap = (const TI*)g.A;
    const TI* Hp = (const TI*)g.Ahead;
    const TI* Bp = (const TI*)g.B;

    // Thread-constant parts of the load coordinates.  A element p of this
    // thread is (row mA + p*ASTEP, k kA) for MK or (row mA, k kA + p*ASTEP)
    // for KM; likewise for B.
    const int mA = AKM ? tid % BM : tid / BK;
    const int kA = AKM ? tid / BM : tid % BK;
    const int nB = BNK ? tid / BK : tid % BN;
    const int kB = BNK ? tid % BK : tid / BN;
    // 32-bit element offsets from the chunk's base pointers (tile-local)
    int offA[LA], offB[LB];
    bool vA[LA], vB[LB];
#pragma unroll
    for (int p = 0; p < LA; ++p) {
        const int r = AKM ? kA + p * ASTEP : mA + p * ASTEP;   // stored row within the chunk/tile
        const int c = AKM ? mA : kA;
        offA[p] = (int)(r * g.lda + c);
        vA[p] = AKM ? (m0 + mA < g.M) : (m0 + mA + p * ASTEP < g.M);
    }
#pragma unroll
    for (int p = 0; p < LB; ++p) {
        const int r = BNK ? nB + p * BSTEP : kB + p * BSTEP;
        const int c = BNK ? kB : nB;
        offB[p] = (int)(r * g.ldb + c);
        vB[p] = BNK ? (n0 + nB + p * BSTEP < g.N) : (n0 + nB < g.N);
    }

    TI ra[LA], rb[LB];

    auto load = [&](int64_t k0) {
        // A
        if (AKM && k0 < g.head_k) {
            // chunk touches the head segment: per-element source selection
#pragma unroll
            for (int p = 0; p < LA; ++p) {
                const int64_t gk = k0 + kA + p * ASTEP, gm = m0 + mA;
                TI v = (TI)0;
                if (vA[p] && gk < kend) {
                    const bool up = g.a_lower && gm > gk;
                    if (!up) v = gk < g.head_k ? Hp[gk * g.ldah + gm] : Ap[(gk - g.head_k) * g.lda + gm];
                }
                ra[p] = v;
            }
        } else {
            const TI* base = AKM ? Ap + (k0 - g.head_k) * g.lda + m0 : Ap + m0 * g.lda + k0;
#pragma unroll
            for (int p = 0; p < LA; ++p) {
                const int64_t gk = AKM ? k0 + kA + p * ASTEP : k0 + kA;
                const int64_t gm = AKM ? m0 + mA : m0 + mA + p * ASTEP;
                const bool ok = vA[p] && gk < kend && !(g.a_lower && (AKM ? gm > gk : gk > gm));
                ra[p] = ok ? base[offA[p]] : (TI)0;
            }
        }
        // B
        const TI* bbase = BNK ? Bp + n0 * g.ldb + k0 : Bp + k0 * g.ldb + n0;
#pragma unroll
        for (int p = 0; p < LB; ++p) {
            const int64_t gk = BNK ? k0 + kB : k0 + kB + p * BSTEP;
            rb[p] = (vB[p] && gk < kend) ? bbase[offB[p]] : (TI)0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < LA; ++p) {
            if (AKM) sA(buf, kA + p * ASTEP)[mA] = ra[p];
            else sA(buf, kA)[mA + p * ASTEP] = ra[p];
        }
#pragma unroll
        for (int p = 0; p < LB; ++p) {
            if (BNK) sB(buf, kB)[nB + p * BSTEP] = rb[p];
            else sB(buf, kB + p * BSTEP)[nB] = rb[p];
        }
    };

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = acc_t{0, 0, 0, 0};

    const int lr = lane >> 4, lc = lane & 15;
    const int64_t nchunk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
    if (nchunk > 0) {
        load(kbeg);
        store(0);
        __syncthreads();
        for (int64_t c = 0; c < nchunk; ++c) {
            const int cur = (int)(c & 1);
            if (c + 1 < nchunk) load(kbeg + (c + 1) * BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                TI a[FM], b[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) a[i] = sA(cur, kk + lr)[wm * WTM + i * 16 + lc];
#pragma unroll
                for (int j = 0; j < FN; ++j) b[j] = sB(cur, kk + lr)[wn * WTN + j * 16 + lc];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = Mfma<TI>::op(a[i], b[j], acc[i][j]);
            }
            if (c + 1 < nchunk) store(cur ^ 1);
            __syncthreads();
        }
    }

    // epilogue
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm * WTM + i * 16 + Mfma<TI>::row(lr, r);
                const int64_t col = n0 + wn * WTN + j * 16 + lc;
                if (row >= g.M || col >= g.N) continue;
                if ((LOWER || g.c_lower) && col > row) continue;
                const double v = (double)acc[i][j][r];
                if (EPI == EPI_SUB) {
                    g.C[row * g.ldc + col] -= v;
                } else if (EPI == EPI_STORE) {
                    g.C[row * g.ldc + col] = v;
                    if (g.Cf) g.Cf[row * g.ldcf + col] = (float)v;
                } else if (EPI == EPI_PARTIAL) {
                    g.C[z * g.pstride + row * g.ldc + col] = v;
                } else if (EPI == EPI_SYMLOW) {
                    if (row >= col) {
                        g.C[row * g.ldc + col] = v;
                        g.C[col * g.ldc + row] = v;
                    }
                } else {  // EPI_PHI
                    g.C[row * g.ldc + col] = v;
                    if (g.Cf) g.Cf[row * g.ldcf + col] = (float)v;
                    g.C2[row * g.ldc2 + col] = row > col ? v : (row == col ? 0.5 * v : 0.0);
                }
            }
}


}  // namespace gpc
