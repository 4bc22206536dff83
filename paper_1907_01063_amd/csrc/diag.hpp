// Register-resident diagonal-block routines shared by the stand-alone kernels
// and the persistent batched kernel (256 threads as a 16 x 16 grid).
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace gpc {

// f(std::integral_constant<int, I>()) for I = B .. E-1, unrolled at compile time.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>());
        static_for<B + 1, E>(f);
    }
}

// 1/sqrt(d) to working precision: the hardware estimate refined by two
// Newton steps y <- y + y (1 - d y^2) / 2 (each one doubles the correct bits).
// NaN for d < 0 and NaN, +inf for d = 0, like 1/sqrt.
__device__ __forceinline__ double rsqrt_refined(double d)
{
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-d * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// ---- tiled factor + inverse with matrix-core products ----------------------
// FP64 MFMA 16x16x4 layouts: the A operand of k-slice kk holds A[l%16][l/16 +
// 4kk] in lane l, the B operand B[l/16 + 4kk][l%16], and the 4 accumulator
// registers hold rows l/16 + 4r of column l%16 ("C layout").  So a tile kept
// in C layout is, register kk for register kk, the B operand of itself; and a
// tile's C-layout registers stored to LDS as [r][lane] read back at
// [kk][lane] as the A operand of that tile's transpose.
typedef double dtile __attribute__((ext_vector_type(4)));

// value selects (a conditional over two lvalues would select their addresses)
template <typename V>
__device__ __forceinline__ V pick(bool c, V a, V b)
{
    return c ? a : b;
}

// orders LDS accesses between the lanes of one wave
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// every lane takes v from lane J of its own row of 16 lanes
template <int J>
__device__ __forceinline__ double row_bcast_f64(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x150 + J, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x150 + J, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// the transpose of a C-layout tile, stored to LDS so that [kk][lane] reads
// give the A operand of the tile itself (T[l%16][l/16 + 4kk])
__device__ __forceinline__ void store_tile_transposed(double* buf, const dtile& t, int lane)
{
    double* q = buf + ((lane & 15) >> 2) * 64 + 16 * (lane & 3) + (lane >> 4);
    static_for<0, 4>([&](auto R_) {
        constexpr int r = decltype(R_)::value;
        q[4 * r] = t[r];
    });
}

__device__ __forceinline__ void store_tile(double* buf, const dtile& t, int lane)
{
    static_for<0, 4>([&](auto R_) {
        constexpr int r = decltype(R_)::value;
        buf[r * 64 + lane] = t[r];
    });
}

// acc + A B, with the A fragments in af and the B fragments in bf
__device__ __forceinline__ dtile mfma_tile(const double (&af)[4], const dtile& bf, dtile acc)
{
    static_for<0, 4>([&](auto KK_) {
        constexpr int kk = decltype(KK_)::value;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[kk], bf[kk], acc, 0, 0, 0);
    });
    return acc;
}

__device__ __forceinline__ void load_frags(const double* buf, int lane, double (&f)[4], double sign)
{
    static_for<0, 4>([&](auto KK_) {
        constexpr int kk = decltype(KK_)::value;
        f[kk] = sign * buf[kk * 64 + lane];
    });
}

__device__ __forceinline__ dtile load_bfrag(const double* buf, int lane)
{
    dtile t;
    static_for<0, 4>([&](auto KK_) {
        constexpr int kk = decltype(KK_)::value;
        t[kk] = buf[kk * 64 + lane];
    });
    return t;
}

// One wave factors the symmetric 16 x 16 tile E (C layout, both triangles)
// and inverts the factor: a column sweep entirely in registers, with the
// column's entries taken from the lanes that hold them (no LDS, no barrier).
// Step j: d = E(j, j); every row rho > j takes E(rho, c) -= E(rho, j) f_c
// with f_c = E(j, c) / d (c != j; E(j, c) is the Schur complement's entry
// for c > j and the running inverse's unscaled row j for c < j) and restarts
// column j as the inverse's column, E(rho, j) = -E(rho, j) / d.  The lanes of
// column j keep its unscaled entries and 1/sqrt(d); the factor's tile is
// formed from them at the end.  On return E holds the inverse Linv (C layout,
// zero above the diagonal), lt the factor's tile (zero above the diagonal);
// the first failed pivot is recorded in info.
__device__ __forceinline__ void factor_tile16(dtile& E, dtile& lt, int lane, int32_t* info, int64_t col0)
{
    // the lane's column and row group, recomputed here so that the per-step
    // lane masks are formed where they are used rather than kept live
    int c, g;
    asm volatile("v_and_b32 %0, 15, %1" : "=v"(c) : "v"(lane));
    asm volatile("v_lshrrev_b32 %0, 4, %1" : "=v"(g) : "v"(lane));
    dtile yr = {0.0, 0.0, 0.0, 0.0};                       // 1/L_rr of the lane's rows
    lt = dtile{0.0, 0.0, 0.0, 0.0};                        // unscaled column c of L
    double ycol = 0.0;                                     // 1/L_cc
    int fail = 0;
    static_for<0, 16>([&](auto J) {
        constexpr int j = decltype(J)::value, jr = j / 4, jg = j % 4;
        const double d = readlane_f64(E[jr], 16 * jg + j);
        const double ejc = __shfl(E[jr], 16 * jg + c, 64);
        double eij[4];
        static_for<jr, 4>([&](auto R_) {
            constexpr int r = decltype(R_)::value;
            eij[r] = row_bcast_f64<j>(E[r]);
        });
        fail = (fail == 0 && !(d > 0.0)) ? j + 1 : fail;
        const double y = rsqrt_refined(d);
        const double rd = y * y;
        const bool own = c == j;
        const double f = pick<double>(own, rd, ejc * rd);
        ycol = pick<double>(own, y, ycol);
        static_for<jr, 4>([&](auto R_) {
            constexpr int r = decltype(R_)::value;
            lt[r] = pick<double>(own, E[r], lt[r]);
            const double upd = pick<double>(own, 0.0, E[r]) - eij[r] * f;
            if constexpr (r == jr) {
                E[r] = pick<double>(g > jg, upd, E[r]);
                yr[r] = pick<double>(g == jg, y, yr[r]);
            } else {
                E[r] = upd;
            }
        });
    });
    if (fail != 0 && lane == 0 && *info == 0) *info = (int32_t)(col0 + fail);
    static_for<0, 4>([&](auto R_) {
        constexpr int r = decltype(R_)::value;
        const int rho = g + 4 * r;
        E[r] = c < rho ? E[r] * yr[r] : (c == rho ? yr[r] : 0.0);
        const double dd = lt[r];
        double l = dd * ycol;                              // sqrt(d), one correction step
        l = fma(0.5 * ycol, fma(-l, l, dd), l);
        lt[r] = c < rho ? dd * ycol : (c == rho ? l : 0.0);
    });
}

// Factor + inverse of one kb x kb diagonal block (kb <= 16 NT) by tiles, the
// "chol" step of section 3.3.1 together with the inverse the panel solve
// multiplies by (section 3.2).  The block is NT x NT tiles of 16 x 16, the
// lower ones (i >= c) held in registers in C layout for the whole kernel:
// wave w < NT/2 owns tile rows w and NT-1-w (NT + 1 tiles: tile (w, c) in
// T[c], tile (NT-1-w, c) in T[NT-c]).  For each tile column p:
//   A  the owner of row p updates tile (p, p) with column p-1 (step C of
//      p-1, taken first), factors and inverts it (one wave), writes L_pp and
//      puts Linv_pp's transpose in LDS; the other owners finish step C of
//      column p-1;                                                 barrier
//   B  owners of rows i > p: L_ip^T = Linv_pp S_ip^T (S_ip = tile (i, p)),
//      written to A and to the panel buffer F[i]; the owner of row p turns
//      its running inverse tiles R_pc (c < p) into the final inverse tiles
//      X_pc = Linv_pp R_pc, and puts them and X_pp = Linv_pp in F[c];  barrier
//   C  owners of rows i > p update every tile (i, c), c <= i:
//        c > p:  S_ic -= L_ip L_cp^T      (Schur complement)
//        c = p:  R_ip  = -L_ip Linv_pp    (restarts as a running inverse tile)
//        c < p:  R_ic -= L_ip X_pc        (forward substitution)
// Rows and columns past kb act as an identity block.  The inverse tiles are
// written at the end, with the strict upper triangles of both outputs zeroed.
// F: NT * 256 doubles, LU: 256 doubles (LDS).  256 threads.
template <int NT>
__device__ void diag_tile_factor_inverse(int kb, double* A, int64_t lda, double* Linv, int64_t ldi,
                                         int32_t* info, int64_t col0, double* F, double* LU)
{
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool active = w < NT / 2;
    const int rowA = w, rowB = NT - 1 - w;             // owned tile rows
    const int np = (kb + 15) >> 4;                     // tile rows holding part of the block
    const int lr = lane >> 4, lc = lane & 15;          // C layout: rows lr + 4r, column lc
    const dtile zero = {0.0, 0.0, 0.0, 0.0};

    dtile T[NT + 1];
    static_for<0, NT + 1>([&](auto I) { T[decltype(I)::value] = zero; });
    // tile (i, c) element (16i + lr + 4r, 16c + lc); the diagonal tiles in
    // full from the lower triangle; identity past kb
    static_for<0, 2>([&](auto RI) {
        constexpr int ri = decltype(RI)::value;
        const int i = ri == 0 ? rowA : rowB;
        static_for<0, NT>([&](auto CC) {
            constexpr int cc = decltype(CC)::value;
            constexpr int idx = ri == 0 ? cc : NT - cc;
            if (active && cc <= i && i < np) {
                static_for<0, 4>([&](auto R_) {
                    constexpr int r = decltype(R_)::value;
                    const int a = 16 * i + lr + 4 * r, b = 16 * cc + lc;
                    const int hi = a > b ? a : b, lo = a > b ? b : a;
                    T[idx][r] = hi < kb ? A[(int64_t)hi * lda + lo] : (a == b ? 1.0 : 0.0);
                });
            }
        });
    });

    for (int p = 0; p < np; ++p) {
        // ---- A: the owner of row p (tile (p, p) is T[p] or T[NT-p])
        const bool pA = active && w == p, pB = active && w == NT - 1 - p;
        if (pA || pB) {
            const int di = pA ? p : NT - p;
            dtile D = zero;
            static_for<0, NT + 1>([&](auto I) {           // selects, not branches, keep T in registers
                const dtile v = T[decltype(I)::value];
                D = pick<dtile>(decltype(I)::value == di, v, D);
            });
            if (p > 0) {
                double ai[4];
                load_frags(F + p * 256, lane, ai, -1.0);
                D = mfma_tile(ai, load_bfrag(F + p * 256, lane), D);
            }
            dtile lt;
            factor_tile16(D, lt, lane, info, col0 + 16 * p);
            static_for<0, 4>([&](auto R_) {
                constexpr int r = decltype(R_)::value;
                const int a = 16 * p + lr + 4 * r, b = 16 * p + lc;
                if (a < kb && b < kb) A[(int64_t)a * lda + b] = lt[r];
            });
            store_tile_transposed(LU, D, lane);
            static_for<0, NT + 1>([&](auto I) {
                const dtile v = T[decltype(I)::value];
                T[decltype(I)::value] = pick<dtile>(decltype(I)::value == di, D, v);
            });
        }
        // ---- the rest of C for column p-1 (one B fragment load serves both rows)
        if (active && p > 0) {
            const int q = p - 1;
            const bool okA = rowA > q && rowA < np, okB = rowB > q && rowB < np;
            double aA[4], aB[4];                                 // -L_iq of the two rows
            load_frags(F + rowA * 256, lane, aA, -1.0);
            load_frags(F + rowB * 256, lane, aB, -1.0);
            static_for<0, NT>([&](auto CC) {
                constexpr int cc = decltype(CC)::value;
                const bool useA = okA && cc <= rowA && !(cc == p && rowA == p);
                const bool useB = okB && cc <= rowB && !(cc == p && rowB == p);
                if (useA || useB) {
                    const dtile b = load_bfrag(F + cc * 256, lane);
                    if (useA) T[cc] = mfma_tile(aA, b, cc == q ? zero : T[cc]);
                    if (useB) T[NT - cc] = mfma_tile(aB, b, cc == q ? zero : T[NT - cc]);
                }
            });
        }
        __syncthreads();
        // ---- B
        if (active) {
            double la[4];
            load_frags(LU, lane, la, 1.0);
            static_for<0, 2>([&](auto RI) {
                constexpr int ri = decltype(RI)::value;
                const int i = ri == 0 ? rowA : rowB;
                if (i > p && i < np) {
                    double* Fi = F + i * 256;
                    dtile sip = zero;                              // tile (i, p)
                    static_for<0, NT>([&](auto CC) {
                        constexpr int cc = decltype(CC)::value;
                        const dtile v = T[ri == 0 ? cc : NT - cc];
                        sip = pick<dtile>(cc == p, v, sip);
                    });
                    store_tile_transposed(Fi, sip, lane);
                    wave_lds_sync();
                    const dtile sb = load_bfrag(Fi, lane);
                    const dtile lt = mfma_tile(la, sb, zero);                   // L_ip^T
                    wave_lds_sync();
                    store_tile(Fi, lt, lane);
                    static_for<0, 4>([&](auto R_) {
                        constexpr int r = decltype(R_)::value;
                        const int a = 16 * i + lc, b = 16 * p + lr + 4 * r;
                        if (a < kb) A[(int64_t)a * lda + b] = lt[r];
                    });
                }
            });
            static_for<0, 2>([&](auto RI) {
                constexpr int ri = decltype(RI)::value;
                if ((ri == 0 ? rowA : rowB) == p) {
                    static_for<0, NT>([&](auto CC) {
                        constexpr int cc = decltype(CC)::value;
                        constexpr int idx = ri == 0 ? cc : NT - cc;
                        if (cc < p) T[idx] = mfma_tile(la, T[idx], zero);
                        if (cc <= p) store_tile(F + cc * 256, T[idx], lane);
                    });
                }
            });
        }
        __syncthreads();
    }
    // the last column's step C has no rows below it

    // write the inverse; zero the strict upper triangles of both outputs
    if (active) {
        static_for<0, 2>([&](auto RI) {
            constexpr int ri = decltype(RI)::value;
            const int i = ri == 0 ? rowA : rowB;
            static_for<0, NT>([&](auto CC) {
                constexpr int cc = decltype(CC)::value;
                constexpr int idx = ri == 0 ? cc : NT - cc;
                if (cc <= i && i < np) {
                    static_for<0, 4>([&](auto R_) {
                        constexpr int r = decltype(R_)::value;
                        const int a = 16 * i + lr + 4 * r, b = 16 * cc + lc;
                        if (a < kb && b < kb) Linv[(int64_t)a * ldi + b] = T[idx][r];
                        if (cc < i) {
                            const int at = 16 * cc + lr + 4 * r, bt = 16 * i + lc;
                            if (bt < kb) {
                                A[(int64_t)at * lda + bt] = 0.0;
                                Linv[(int64_t)at * ldi + bt] = 0.0;
                            }
                        }
                    });
                }
            });
        });
    }
}

// Factor + inverse of one diagonal block held in registers element-wise,
// columns eliminated four at a time (the persistent batched kernel's form).
// Thread (ty, tx) of a 16 x 16 grid owns the elements (i, c) = (ty + 16a, tx + 16b)
// with a >= b (the lower triangle, up to 36 per thread) in E[a][b] for the
// whole kernel.  Columns are eliminated four at a time (J = j .. j+3), one
// barrier per group:
//   publish  the owners of the group's columns put their Schur-complement
//            entries P_r = E(r, J) (zero above the diagonal) in colbuf; the
//            owners of the group's rows put their running inverse entries
//            Q_c = E(J, c), c < j, in rowbuf;                          barrier
//   update   every thread factors the 4 x 4 diagonal block S = l l^T itself
//            (refined 1/sqrt for the pivots; a failed pivot is recorded) and
//            forms Y = l^-1, then for the rows i and columns c it owns
//            L(i, J) = P_i Y^T and F(c) = Y V_c, with V_c = P_c below the
//            group, Q_c left of it and the unit vector inside it, so that F(c)
//            is L(c, J) below the group (Schur complement), the final rows J of
//            the inverse left of it, and Y's columns inside it (inverse by
//            forward substitution).  Rows below the group take
//            E(i, c) -= L(i, J) F(c) (the group's own columns restart at 0 as
//            inverse columns); rows of the group finish their inverse row:
//            E(i, c) = l_ii F_i(c), c < i.
// so the factor of section 3.3.1's diagonal step and its inverse (used by the
// panel solve) come out of the same sweep.  E(i, c), c < i, ends as the
// inverse's entry scaled by l_ii; the inverse is written once at the end and
// the columns of L as each group is done.  The broadcast buffers alternate
// between groups (a thread that publishes group g + 2 has passed the barrier
// of group g + 1, which every thread reaches only after its update with group
// g).  LDS use is small (about 17 KB at NA = 8), so the kernel can share a CU
// with the product kernels that run beside it.  Columns past kb act as an
// identity block (unit pivots, zero coupling).
// NA: number of 16-row groups (block edge up to 16 * NA); 256 threads.
// colbuf, rowbuf: 2 * 4 * 16 * NA doubles; rls: 16 * NA doubles (all LDS).
// A: byte offsets of a 16 NA row band fit in 31 bits.
template <int NA>
__device__ void diag_factor_inverse_g4(int kb, double* A, int64_t lda, double* Linv, int64_t ldi, int32_t* info,
                                    int64_t col0, double* colbuf, double* rowbuf, double* rls)
{
    constexpr int NB = 16 * NA, G = 4;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc(A, (short)0, 0x7fffffff, 0x00020000);

    double E[NA][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = ty + 16 * a, c = tx + 16 * b;
            E[a][b] = (i < kb && c <= i) ? A[i * lda + c] : 0.0;
        }
    // wait for the block's loads here, once: otherwise the wait for them sits
    // inside the column loop, where it also waits for every store of L issued
    // by the previous columns
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    // byte offset of row ty + 16a of A
    uint32_t rowoff[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) rowoff[a] = (uint32_t)((ty + 16 * a) * lda) * 8u;

    // block columns aj = 0 .. NA-1 with aj a compile-time constant, so that
    // every index into E stays static and E stays in registers
    static_for<0, NA>([&](auto ajc) {
        constexpr int aj = decltype(ajc)::value;
        if (aj * 16 >= kb) return;
        for (int rg = 0; rg < 16 / G; ++rg) {
            const int j = aj * 16 + rg * G;
            if (j >= kb) break;
            double* cb = colbuf + ((j / G) & 1) * NB * G;
            double* rb = rowbuf + ((j / G) & 1) * NB * G;
            const int tc = tx - G * rg;   // group column of this thread's block-aj column (0..3 if in J)
            const int tr = ty - G * rg;   // group row of this thread's block-aj row
            // publish
            if (tc >= 0 && tc < G) {
#pragma unroll
                for (int a = aj; a < NA; ++a) {
                    const int r = ty + 16 * a;
                    cb[r * G + tc] = r >= j + tc ? E[a][aj] : 0.0;
                }
            }
            if (tr >= 0 && tr < G) {
#pragma unroll
                for (int b = 0; b <= aj; ++b) {
                    const int c = tx + 16 * b;
                    rb[c * G + tr] = c < j ? E[aj][b] : 0.0;
                }
            }
            __syncthreads();

            // 4 x 4 diagonal block: S = l l^T, Y = l^-1 (every thread)
            double S[G][G], l[G][G], y[G], Y[G][G];
#pragma unroll
            for (int s2 = 0; s2 < G; ++s2)
#pragma unroll
                for (int t = 0; t <= s2; ++t) S[s2][t] = cb[(j + s2) * G + t];
#pragma unroll
            for (int t = 0; t < G; ++t) {
                double dt = S[t][t];
#pragma unroll
                for (int u = 0; u < t; ++u) dt -= l[t][u] * l[t][u];
                const bool valid = j + t < kb;
                if (tid == 0 && valid && !(dt > 0.0) && *info == 0) *info = (int32_t)(col0 + j + t + 1);
                dt = valid ? dt : 1.0;
                y[t] = rsqrt_refined(dt);
                double lt = dt * y[t];
                l[t][t] = fma(0.5 * y[t], fma(-lt, lt, dt), lt);
#pragma unroll
                for (int s2 = t + 1; s2 < G; ++s2) {
                    double v = S[s2][t];
#pragma unroll
                    for (int u = 0; u < t; ++u) v -= l[s2][u] * l[t][u];
                    l[s2][t] = v * y[t];
                }
            }
#pragma unroll
            for (int t = 0; t < G; ++t) {
                Y[t][t] = y[t];
#pragma unroll
                for (int s2 = 0; s2 < t; ++s2) {
                    double v = 0.0;
#pragma unroll
                    for (int u = s2; u < t; ++u) v += l[t][u] * Y[u][s2];
                    Y[t][s2] = -y[t] * v;
                }
            }
            if (tid < G && j + tid < kb) rls[j + tid] = tid == 0 ? y[0] : tid == 1 ? y[1] : tid == 2 ? y[2] : y[3];

            // L(i, J) for the owned rows (a >= aj), F(c) for the owned columns
            double Lr[NA][G], F[NA][G];
#pragma unroll
            for (int a = aj; a < NA; ++a) {
                double P[G];
#pragma unroll
                for (int s2 = 0; s2 < G; ++s2) P[s2] = cb[(ty + 16 * a) * G + s2];
#pragma unroll
                for (int t = 0; t < G; ++t) {
                    double v = 0.0;
#pragma unroll
                    for (int s2 = 0; s2 <= t; ++s2) v += Y[t][s2] * P[s2];
                    Lr[a][t] = v;
                }
            }
#pragma unroll
            for (int b = 0; b < NA; ++b) {
                const int c = tx + 16 * b;
                double V[G];
#pragma unroll
                for (int s2 = 0; s2 < G; ++s2) {
                    if (b < aj) V[s2] = rb[c * G + s2];
                    else if (b > aj) V[s2] = cb[c * G + s2];
                    else V[s2] = c >= j + G ? cb[c * G + s2] : (c < j ? rb[c * G + s2] : (c - j == s2 ? 1.0 : 0.0));
                }
#pragma unroll
                for (int t = 0; t < G; ++t) {
                    double v = 0.0;
#pragma unroll
                    for (int s2 = 0; s2 <= t; ++s2) v += Y[t][s2] * V[s2];
                    F[b][t] = v;
                }
            }
            // columns J of L, written by their owners
            if (tc >= 0 && tc < G && j + tc < kb) {
#pragma unroll
                for (int a = aj; a < NA; ++a) {
                    const int i = ty + 16 * a;
                    if (i >= j + tc && i < kb) {
                        const double v = tc == 0 ? Lr[a][0] : tc == 1 ? Lr[a][1] : tc == 2 ? Lr[a][2] : Lr[a][3];
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                                              ra, (int)(rowoff[a] + 8u * (j + tc)), 0, 0);
                    }
                }
            }
            // updates: rows below the group; rows of the group finish their inverse row
#pragma unroll
            for (int a = aj; a < NA; ++a) {
                const int i = ty + 16 * a;
                const bool below = a > aj || tr >= G;
                const bool inJ = a == aj && tr >= 0 && tr < G;
                double lii = 0.0;
                if (a == aj) lii = tr == 0 ? l[0][0] : tr == 1 ? l[1][1] : tr == 2 ? l[2][2] : l[3][3];
#pragma unroll
                for (int b = 0; b <= a; ++b) {
                    const int c = tx + 16 * b;
                    if (below) {
                        double v = (b == aj && tc >= 0 && tc < G) ? 0.0 : E[a][b];
#pragma unroll
                        for (int t = 0; t < G; ++t) v -= Lr[a][t] * F[b][t];
                        E[a][b] = v;
                    } else if (inJ && c < i) {
                        const double f = tr == 0 ? F[b][0] : tr == 1 ? F[b][1] : tr == 2 ? F[b][2] : F[b][3];
                        E[a][b] = lii * f;
                    }
                }
            }
        }
    });
    __syncthreads();

    // write out the inverse (row i scaled by 1/l_ii) and zero both upper halves
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = ty + 16 * a, c = tx + 16 * b;
            if (i < kb && c <= i) Linv[i * ldi + c] = c < i ? E[a][b] * rls[i] : rls[i];
        }
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        if (c > r) {
            A[r * lda + c] = 0.0;
            Linv[r * ldi + c] = 0.0;
        }
    }
}


// Inverse X = L^-1 of a lower-triangular block (edge kb <= 16 * NA) read from
// global memory; the block sits in LDS (Ls, pitch 16*NA + 1) and thread
// (ty, tx) keeps the inverse's entries (ty + 16a, tx + 16b), a >= b, in
// registers.  Step j: the owners of row j publish the final row
// X_jc = E(j,c) / L_jj (c < j) and X_jj = 1 / L_jj; then every thread does
// E(i,c) -= L_ij X_jc for i > j, c <= j (forward substitution on all
// columns at once).  X is written with leading dimension ldx, upper := 0.
template <int NA>
__device__ void diag_inverse(int kb, const double* L, int64_t ldl, double* X, int64_t ldx, double* Ls,
                             double* rowbuf)
{
    constexpr int P = 16 * NA + 1;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    // 16 loads per thread issued before their stores to LDS
    for (int base = 0; base < kb * kb; base += 16 * 256) {
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int idx = base + tid + 256 * k;
            const int r = idx / kb, c = idx % kb;
            v[k] = (idx < kb * kb && c <= r) ? L[r * ldl + c] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int idx = base + tid + 256 * k;
            const int r = idx / kb, c = idx % kb;
            if (idx < kb * kb) {
                Ls[r * P + c] = v[k];
                if (c > r) X[r * ldx + c] = 0.0;
            }
        }
    }
    double E[NA][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b)
            E[a][b] = (ty + 16 * a == tx + 16 * b) ? 1.0 : 0.0;
    __syncthreads();
#pragma unroll
    for (int aj = 0; aj < NA; ++aj) {
        if (aj * 16 >= kb) break;
        for (int rj = 0; rj < 16; ++rj) {
            const int j = aj * 16 + rj;
            if (j >= kb) break;
            const double rl = 1.0 / Ls[j * P + j];
            if (ty == rj) {
#pragma unroll
                for (int b = 0; b <= aj; ++b) {
                    const int c = tx + 16 * b;
                    if (c <= j) {
                        const double xh = E[aj][b] * rl;
                        rowbuf[c] = xh;
                        X[j * ldx + c] = xh;
                    }
                }
            }
            __syncthreads();
            double g[NA], f[NA];
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int i = ty + 16 * a;
                g[a] = (i > j && i < kb) ? Ls[i * P + j] : 0.0;
            }
#pragma unroll
            for (int b = 0; b < NA; ++b) {
                const int c = tx + 16 * b;
                f[b] = c <= j ? rowbuf[c] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    E[a][b] -= g[a] * f[b];
            __syncthreads();
        }
    }
}

}  // namespace gpc
