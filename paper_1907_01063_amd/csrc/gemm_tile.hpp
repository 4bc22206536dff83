// MFMA tile body shared by the stand-alone GEMM kernels and the persistent
// batched kernel.  See gemm.hip for the scheme.
#pragma once

#include <type_traits>

#include "internal.hpp"
#include "tile_order.hpp"

namespace gpc {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4v acc_t;
    typedef double elem_t;
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lr, int r) { return lr + 4 * r; }
};
template <> struct Mfma<float> {
    typedef f4v acc_t;
    typedef float elem_t;
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lr, int r) { return 4 * lr + r; }
};

// Operand loads go through buffer resources: a uniform base per chunk plus a
// thread-constant 32-bit byte offset.  An element outside the operand gets an
// offset past the resource's range, which the hardware returns as zero, so
// the loads need no branches and no 64-bit addresses.
constexpr uint32_t kOffOut = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t operand_rsrc(const void* base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000);
}
template <typename T> __device__ __forceinline__ T buffer_ld(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ double buffer_ld<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ float buffer_ld<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}


template <typename TI, int BM, int BN, int BK>
struct TileLds {
    static constexpr int PAD = sizeof(TI) == 8 ? 2 : 4;
    static constexpr int elems = 2 * BK * (BM + PAD) + 2 * BK * (BN + PAD);
};

// One BM x BN output tile (tile row tm, tile column tn, split slice z) computed
// by the whole workgroup (WM x WN waves).  lds: TileLds<...>::elems elements.
// Ends with all LDS reads done, so calls may follow each other directly.
// TG: element type of A and B in memory (default TI); loads convert to TI.
template <typename TI, int BM, int BN, int BK, int WM, int WN, bool AKM, bool BNK, int EPI, bool LOWER,
          typename TG = TI>
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

    typedef TI RowA[BM + PAD];
    typedef TI RowB[BN + PAD];
    RowA* sA0 = (RowA*)lds;
    RowB* sB0 = (RowB*)(lds + 2 * BK * (BM + PAD));
    auto sA = [&](int buf, int kk) -> RowA& { return sA0[buf * BK + kk]; };
    auto sB = [&](int buf, int kk) -> RowB& { return sB0[buf * BK + kk]; };

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN;

    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int64_t kbeg = z * g.kchunk;
    // staircase: the tile's rows end their inner dimension at (m0 / kstep + 1) kstep (uniform per tile)
    const int64_t kend = min(g.kstep > 0 ? min(g.K, (m0 / g.kstep + 1) * g.kstep) : g.K, kbeg + g.kchunk);

    // no __restrict__: the in-place panel products write the rows they read
    const TG* Ap = (const TG*)g.A;
    const TG* Hp = (const TG*)g.Ahead;
    const TG* Bp = (const TG*)g.B;

    // Thread-constant parts of the load coordinates.  A element p of this
    // thread is (row mA + p*ASTEP, k kA) for MK or (row mA, k kA + p*ASTEP)
    // for KM; likewise for B.
    const int mA = AKM ? tid % BM : tid / BK;
    const int kA = AKM ? tid / BM : tid % BK;
    const int nB = BNK ? tid / BK : tid % BN;
    const int kB = BNK ? tid % BK : tid / BN;
    // 32-bit byte offsets from the chunk's base pointers (tile-local); rows
    // (MK/NK) or columns (KM/KN) outside the operand get kOffOut once here
    uint32_t offA[LA], offB[LB];
#pragma unroll
    for (int p = 0; p < LA; ++p) {
        const int r = AKM ? kA + p * ASTEP : mA + p * ASTEP;   // stored row within the chunk/tile
        const int c = AKM ? mA : kA;
        const bool v = AKM ? (m0 + mA < g.M) : (m0 + mA + p * ASTEP < g.M);
        offA[p] = v ? (uint32_t)(r * g.lda + c) * (uint32_t)sizeof(TG) : kOffOut;
    }
#pragma unroll
    for (int p = 0; p < LB; ++p) {
        const int r = BNK ? nB + p * BSTEP : kB + p * BSTEP;
        const int c = BNK ? kB : nB;
        const bool v = BNK ? (n0 + nB + p * BSTEP < g.N) : (n0 + nB < g.N);
        offB[p] = v ? (uint32_t)(r * g.ldb + c) * (uint32_t)sizeof(TG) : kOffOut;
    }

    TI ra[LA], rb[LB];

    // k-row and lower-mask tests against uniform bounds: per thread only kA,
    // kB and (mA - kA) live in registers, whatever LA and LB are
    const int dA = mA - kA;
    auto load = [&](int64_t k0) {
        const int krem = (int)(kend - k0);          // k rows of this chunk in range
        const int dmk = (int)(k0 - m0);             // a_lower: element (m, k) masked where m - k > dmk (KM)
        const bool alow = g.a_lower != 0;
        // A
        if (AKM && k0 < g.head_k) {
            // KM chunk that starts in the head segment: k < head_k reads Ahead
            // (ld ldah), the rest reads A from its first row
            const int hrem = (int)(g.head_k - k0);
            const auto rh = operand_rsrc(Hp + k0 * g.ldah + m0);
            uint32_t oh[LA];
            bool in[LA];
#pragma unroll
            for (int p = 0; p < LA; ++p) {
                const int kk = kA + p * ASTEP;
                in[p] = (offA[p] != kOffOut) & (kk < krem) & !(alow & (dA - p * ASTEP > dmk));
                oh[p] = (in[p] & (kk < hrem)) ? (uint32_t)(kk * g.ldah + mA) * (uint32_t)sizeof(TG) : kOffOut;
            }
            if (hrem >= BK) {            // whole chunk in the head
#pragma unroll
                for (int p = 0; p < LA; ++p) ra[p] = (TI)buffer_ld<TG>(rh, oh[p]);
            } else {                     // chunk straddles the end of the head
                const auto rm = operand_rsrc(Ap + m0);
                TI h[LA];
#pragma unroll
                for (int p = 0; p < LA; ++p) {
                    const int kk = kA + p * ASTEP;
                    const uint32_t om = (in[p] & (kk >= hrem)) ? (uint32_t)((kk - hrem) * g.lda + mA) * (uint32_t)sizeof(TG) : kOffOut;
                    h[p] = (TI)buffer_ld<TG>(rh, oh[p]);
                    ra[p] = (TI)buffer_ld<TG>(rm, om);
                }
#pragma unroll
                for (int p = 0; p < LA; ++p) ra[p] += h[p];   // one of the two is zero
            }
        } else {
            // offsets selected first, then all loads issued back to back
            uint32_t o[LA];
#pragma unroll
            for (int p = 0; p < LA; ++p) {
                const bool ok = AKM ? (kA < krem - p * ASTEP) & !(alow & (dA > dmk + p * ASTEP))
                                    : (kA < krem) & !(alow & (-dA > p * ASTEP - dmk));
                o[p] = ok ? offA[p] : kOffOut;
            }
            const auto rs = operand_rsrc(AKM ? Ap + (k0 - g.head_k) * g.lda + m0 : Ap + m0 * g.lda + k0);
#pragma unroll
            for (int p = 0; p < LA; ++p) ra[p] = (TI)buffer_ld<TG>(rs, o[p]);
        }
        // B
        uint32_t o[LB];
#pragma unroll
        for (int p = 0; p < LB; ++p) o[p] = (BNK ? kB < krem : kB < krem - p * BSTEP) ? offB[p] : kOffOut;
        const auto rs = operand_rsrc(BNK ? Bp + n0 * g.ldb + k0 : Bp + k0 * g.ldb + n0);
#pragma unroll
        for (int p = 0; p < LB; ++p) rb[p] = (TI)buffer_ld<TG>(rs, o[p]);
    };
    // FP64 subtract (add): the accumulators start at C and the MFMAs are fed
    // -A (A), so they form C - A B (C + A B) directly and the epilogue only
    // writes.  The C loads are issued right after the first operand chunk's,
    // so their latency overlaps it instead of following the last MFMA.
    constexpr bool kAcc = EPI == EPI_SUB || EPI == EPI_ADD;
    constexpr bool kFold = kAcc && sizeof(TI) == 8;
    constexpr bool kNegA = kFold && EPI == EPI_SUB;
    // FP32 subtract from FP64 C, small tiles: C is read into FP64 registers at
    // the same point (there is room for them in a 64 x 64 tile) and the
    // epilogue writes C - A B without a read of its own
    constexpr bool kPre = kAcc && sizeof(TI) == 4 && FM * FN <= 4;
    // FP32 subtract, larger tiles: the same FP64 copy of C is read just
    // before the last k-chunk, when the staging registers are free, so its
    // latency overlaps that chunk's MFMAs
    constexpr bool kLate = kAcc && sizeof(TI) == 4 && !kPre;
    constexpr bool kC = kPre || kLate;
    typedef typename Mfma<TI>::acc_t acc_t;
    acc_t acc[FM][FN];
    double cpre[kC ? FM : 1][kC ? FN : 1][4];
    const int lr = lane >> 4, lc = lane & 15;
    auto load_c = [&]() {
        const auto rc = operand_rsrc(g.C + m0 * g.ldc + n0);
        const uint32_t ldc8 = (uint32_t)g.ldc * 8u;
        const bool lowc = LOWER || g.c_lower;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm * WTM + i * 16 + Mfma<TI>::row(lr, r);
                    const int col = wn * WTN + j * 16 + lc;
                    const bool in = (m0 + row < g.M) & (n0 + col < g.N) & !(lowc & (n0 + col > m0 + row));
                    const double cv = buffer_ld<double>(rc, in ? (uint32_t)row * ldc8 + (uint32_t)col * 8u : kOffOut);
                    if (kC) cpre[kC ? i : 0][kC ? j : 0][r] = cv;
                    else acc[i][j][r] = (typename Mfma<TI>::elem_t)cv;
                }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < LA; ++p) {
            const TI v = kNegA ? -ra[p] : ra[p];
            if (AKM) sA(buf, kA + p * ASTEP)[mA] = v;
            else sA(buf, kA)[mA + p * ASTEP] = v;
        }
#pragma unroll
        for (int p = 0; p < LB; ++p) {
            if (BNK) sB(buf, kB)[nB + p * BSTEP] = rb[p];
            else sB(buf, kB + p * BSTEP)[nB] = rb[p];
        }
    };

    if (!kFold) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = acc_t{0, 0, 0, 0};
    }

    const int64_t nchunk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
    // LDS layouts.  Register path: both operands k-major, sA[k][m] and
    // sB[k][n] (pitch BM + PAD).  Direct path (16-byte lane loads that go
    // straight from memory into LDS, no register staging):
    //  - an MK or NK operand is stored row-major, BK k values (128 B) per row,
    //    with the row's 16-byte groups permuted by (row >> 1) & 7, so that the
    //    16 rows one MFMA operand fetch touches fall into distinct banks;
    //  - a KM or KN operand stays k-major: FP64 k-rows are 1 KB (one wave
    //    load each, padded pitch as in the register path); FP32 k-rows are
    //    512 B, stored unpadded two per wave load, with the 16-byte groups of
    //    row k permuted by (k & 3) << 2 (the four k-rows of one fetch then
    //    sit 64 B apart in the banks).
    // Direct loads carry no sign flip, so the subtracting form negates A at
    // the fragment read instead.
    constexpr int VE = 16 / (int)sizeof(TI);   // elements per 16-byte group
    const int sw = (lc >> 1) & 7;             // group permutation of the MK/NK rows this lane reads
    auto frag = [&](const TI* buf, int k, int r, bool kmajor_padded, bool rowmajor) -> TI {
        if (rowmajor) return buf[r * BK + (((k / VE) ^ sw) * VE) + (k % VE)];
        if (kmajor_padded) return buf[k * (BM + PAD) + r];
        return buf[k * BM + (((r >> 2) ^ ((k & 3) << 2)) << 2) + (r & 3)];   // FP32 k-major, permuted
    };
    auto compute = [&](int cur, auto dir_tag) {
        constexpr bool dir = decltype(dir_tag)::value;
        const TI* bufA = &sA(cur, 0)[0];
        const TI* bufB = &sB(cur, 0)[0];
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int k = kk + lr;
            TI a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int r = wm * WTM + i * 16 + lc;
                if (dir) {
                    const TI x = frag(bufA, k, r, AKM && sizeof(TI) == 8, !AKM);
                    a[i] = kNegA ? -x : x;
                } else {
                    a[i] = sA(cur, k)[r];
                }
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int c = wn * WTN + j * 16 + lc;
                b[j] = dir ? frag(bufB, k, c, !BNK && sizeof(TI) == 8, BNK) : sB(cur, k)[c];
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = Mfma<TI>::op(a[i], b[j], acc[i][j]);
        }
    };
    typedef std::integral_constant<bool, true> DirectTag;
    typedef std::integral_constant<bool, false> RegTag;

    // direct path: 128 x 128 tiles of 8 waves whose k-chunk is 128 B per
    // row-major row, 16-byte aligned rows, no per-element masks; k-major
    // operands must cover whole tile rows (16-byte groups inside the operand,
    // FP32 head rows in pairs), row-major k ranges a whole number of groups
    // (groups never straddle the k end)
    constexpr bool kDirectShape =
        sizeof(TI) == sizeof(TG) && BM == 128 && BN == 128 && NT == 512 && BK * sizeof(TI) == 128;
    bool direct = false;
    if (kDirectShape && nchunk > 0 && g.a_lower == 0) {
        const bool kgroups = ((kend - kbeg) % VE) == 0;
        const bool okA = ((uintptr_t)Ap & 15) == 0 && (g.lda % VE) == 0 &&
                         (AKM ? (m0 + BM <= g.M &&
                                 (g.head_k == 0 || (((uintptr_t)Hp & 15) == 0 && (g.ldah % VE) == 0 &&
                                                    (sizeof(TI) == 8 || (g.head_k & 1) == 0))))
                              : kgroups);
        const bool okB = ((uintptr_t)Bp & 15) == 0 && (g.ldb % VE) == 0 && (BNK ? kgroups : n0 + BN <= g.N);
        direct = okA && okB;
    }
    if (kDirectShape && direct) {
        typedef __attribute__((address_space(3))) void lds_void;
        // MK / NK: wave w fills rows 8w .. 8w+7 and 64+8w .. 64+8w+7; lane l
        // takes row 8w + l/8 (+64) and stores its group l%8, which holds the
        // operand's k group (l%8) ^ ((row >> 1) & 7)
        const int rr = 8 * wave + (lane >> 3);
        const int pp = (lane & 7) ^ ((rr >> 1) & 7);    // same for rr + 64
        // FP32 KM / KN: wave w fills k-rows 2w, 2w+1 and 16+2w, 16+2w+1; lane l
        // takes k-row 2w + l/32 (+16) and stores group l%32, which holds the
        // operand's group (l%32) ^ ((k & 3) << 2)
        const int kq = 2 * wave + (lane >> 5);
        const int gq = (lane & 31) ^ ((kq & 3) << 2);  // same for kq + 16
        auto issue = [&](int64_t k0, int buf) {
            const int krem = (int)(kend - k0);
            TI* dA = &sA(buf, 0)[0];
            TI* dB = &sB(buf, 0)[0];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (AKM && sizeof(TI) == 8) {
                    const int kk = wave + 8 * h;
                    const int64_t gk = k0 + kk;
                    const TG* base = gk < g.head_k ? Hp + gk * g.ldah + m0 : Ap + (gk - g.head_k) * g.lda + m0;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(operand_rsrc(base), (lds_void*)&sA(buf, kk)[0], 16,
                                                             kk < krem ? (uint32_t)lane * 16u : kOffOut, 0, 0, 0);
                } else if (AKM) {
                    const int kr = 2 * wave + 16 * h;          // first k-row of this load (even)
                    const int64_t gk = k0 + kr;                 // k-rows gk, gk+1 come from the same segment
                    const bool head = gk < g.head_k;
                    const TG* base = head ? Hp + gk * g.ldah + m0 : Ap + (gk - g.head_k) * g.lda + m0;
                    const int64_t ld = head ? g.ldah : g.lda;
                    const int kl = lane >> 5;                   // 0 or 1
                    const uint32_t off =
                        kr + kl < krem ? (uint32_t)(kl * ld + 4 * gq) * (uint32_t)sizeof(TG) : kOffOut;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(operand_rsrc(base), (lds_void*)(dA + kr * BM), 16, off,
                                                             0, 0, 0);
                } else {
                    const int r = rr + 64 * h;
                    const uint32_t off = ((m0 + r < g.M) & (VE * pp < krem))
                                             ? (uint32_t)(r * g.lda + VE * pp) * (uint32_t)sizeof(TG) : kOffOut;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(operand_rsrc(Ap + m0 * g.lda + k0),
                                                             (lds_void*)(dA + (8 * wave + 64 * h) * BK), 16, off, 0, 0,
                                                             0);
                }
                if (!BNK && sizeof(TI) == 8) {
                    const int kk = wave + 8 * h;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(operand_rsrc(Bp + (k0 + kk) * g.ldb + n0),
                                                             (lds_void*)&sB(buf, kk)[0], 16,
                                                             kk < krem ? (uint32_t)lane * 16u : kOffOut, 0, 0, 0);
                } else if (!BNK) {
                    const int kr = 2 * wave + 16 * h;
                    const int kl = lane >> 5;
                    const uint32_t off =
                        kr + kl < krem ? (uint32_t)(kl * g.ldb + 4 * gq) * (uint32_t)sizeof(TG) : kOffOut;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(operand_rsrc(Bp + (k0 + kr) * g.ldb + n0),
                                                             (lds_void*)(dB + kr * BN), 16, off, 0, 0, 0);
                } else {
                    const int r = rr + 64 * h;
                    const uint32_t off = ((n0 + r < g.N) & (VE * pp < krem))
                                             ? (uint32_t)(r * g.ldb + VE * pp) * (uint32_t)sizeof(TG) : kOffOut;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(operand_rsrc(Bp + n0 * g.ldb + k0),
                                                             (lds_void*)(dB + (8 * wave + 64 * h) * BK), 16, off, 0, 0,
                                                             0);
                }
            }
        };
        issue(kbeg, 0);
        if (kFold || kPre) load_c();
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this thread's LDS loads landed
        __syncthreads();
        int64_t c = 0;
        for (; c + 1 < nchunk; ++c) {
            const int cur = (int)(c & 1);
            issue(kbeg + (c + 1) * BK, cur ^ 1);
            compute(cur, DirectTag());
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __syncthreads();
        }
        if (kLate) load_c();
        compute((int)(c & 1), DirectTag());
        __syncthreads();
    } else if (nchunk > 0) {
        load(kbeg);
        if (kFold || kPre) load_c();
        store(0);
        __syncthreads();
        // the last chunk is peeled off, so every iteration's loads are
        // consumed by its own LDS stores (no load is ever pending across the
        // back edge, and the loads of one chunk are issued back to back)
        int64_t c = 0;
        for (; c + 1 < nchunk; ++c) {
            const int cur = (int)(c & 1);
            load(kbeg + (c + 1) * BK);
            compute(cur, RegTag());
            store(cur ^ 1);
            __syncthreads();
        }
        if (kLate) load_c();
        compute((int)(c & 1), RegTag());
        __syncthreads();
    } else if (kFold || kC) {
        load_c();
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
                    if (kFold) g.C[row * g.ldc + col] = v;
                    else if (kC) g.C[row * g.ldc + col] = cpre[kC ? i : 0][kC ? j : 0][r] - v;
                    else g.C[row * g.ldc + col] -= v;
                } else if (EPI == EPI_ADD) {
                    if (kFold) g.C[row * g.ldc + col] = v;
                    else if (kC) g.C[row * g.ldc + col] = cpre[kC ? i : 0][kC ? j : 0][r] + v;
                    else g.C[row * g.ldc + col] += v;
                } else if (EPI == EPI_STORE) {
                    g.C[row * g.ldc + col] = g.negate ? -v : v;
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
