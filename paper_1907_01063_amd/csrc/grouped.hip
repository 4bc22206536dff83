// Many covariance matrices of uneven order, factored and differentiated by
// block steps taken by all members at once ("grouped" schedule of the batched
// entry points).
//
// The persistent kernel (batched.hip) gives each matrix to one workgroup, so
// the largest members set the makespan.  Here every step of the blocked
// algorithms of section 3.3 is one launch over all members that still have
// that step: the diagonal-block factor (one workgroup per member), the panel
// product and the trailing update (one workgroup per 64 x 64 output tile of
// every member; steps in pairs, the first updating only the next block's
// columns and the second the rest with both panels, inner dimension 128); the
// reverse sweep likewise (diagonal inverse,
// panel product, left update, the split products of the diagonal step, row
// update).  Member i runs its own step s at launch step s: in the factor its
// block s from the top, in the reverse sweep its block s from the bottom, so
// small members drop out early and the large ones keep every CU busy.  No
// workgroup waits for another; launches are ordered by the stream.  Results
// of a member do not depend on the other members (same arithmetic, same
// order).
#include <string.h>

#include <algorithm>
#include <vector>

#include "diag.hpp"
#include "gemm_tile.hpp"

namespace gpc {
namespace {

constexpr int kGB = 64;       // block size of the grouped schedule
constexpr int kPSlices = 8;   // most k-slices of P = Cbar^T C per member
// 64 x 64 scratch blocks per member: X, the slices of P, W, S, T, M
constexpr int kScrX = 0, kScrP = 1, kScrW = kScrP + kPSlices, kScrS = kScrW + 1, kScrT = kScrS + 1,
              kScrM = kScrT + 1, kGScr = kScrM + 1;

struct GTile {
    int32_t arg, tm, tn, z;   // z: k-slice of a split product
};
struct GDiag {   // factor + inverse of a diagonal block / inverse alone / W = tril(Dbar - sum of P slices)
    double* A;
    const double* P;   // W step: the slices of P, kGB^2 apart (nullptr: none)
    double* X;         // inverse (factor, inverse) / W (W step)
    int32_t* info;
    int64_t lda;
    int64_t col0;
    int32_t kb;
    int32_t np;        // W step: number of slices of P
};
struct GZero {
    double* A;
    int64_t n;
};

template <typename TI, bool AKM, bool BNK, int EPI, bool LOWER>
__global__ void __launch_bounds__(256) grouped_gemm_kernel(const GemmArgs* args, const GTile* tiles)
{
    __shared__ TI lds[TileLds<TI, 64, 64, 16>::elems];
    // XCD x takes the x-th contiguous range of tiles (a member's tiles are
    // contiguous, so they share their operand panels in that XCD's L2)
    const int nwg = gridDim.x, w = blockIdx.x, per = nwg / 8;
    const int t = w < per * 8 ? (w % 8) * per + w / 8 : w;
    const GTile tt = tiles[t];
    const GemmArgs g = args[tt.arg];
    gemm_tile<TI, 64, 64, 16, 2, 2, AKM, BNK, EPI, LOWER, double>(g, tt.tm, tt.tn, 0, lds);
}

// Two products of one block step in one launch: workgroups [0, n1) take the
// tiles of list 1 (the k-slices of P = Cbar^T C, long inner dimension, so
// first), the rest those of list 2 (Bbar -= Cbar R, FP64 or FP32 products).
template <typename TU>
__global__ void __launch_bounds__(256) grouped_p_bbar_kernel(const GemmArgs* a1, const GTile* t1, int n1,
                                                             const GemmArgs* a2, const GTile* t2)
{
#if defined(__HIP_DEVICE_COMPILE__)   // the host pass needs only the launch stub
    __shared__ double lds[TileLds<double, 64, 64, 16>::elems];
    const int nwg = gridDim.x, w = blockIdx.x, per = nwg / 8;
    const int t = w < per * 8 ? (w % 8) * per + w / 8 : w;
    if (t < n1) {
        const GTile tt = t1[t];
        const GemmArgs g = a1[tt.arg];
        gemm_tile<double, 64, 64, 16, 2, 2, true, false, EPI_PARTIAL, false, double>(g, tt.tm, tt.tn, tt.z, lds);
    } else {
        const GTile tt = t2[t - n1];
        const GemmArgs g = a2[tt.arg];
        gemm_tile<TU, 64, 64, 16, 2, 2, false, false, EPI_SUB, false, double>(g, tt.tm, tt.tn, 0, (TU*)lds);
    }
#endif
}

// The diagonal step of one member per workgroup: W = tril(Dbar - P),
// S = sym(D^T W), T = S X, M = X^T T with Dbar <- Phi(M); each product one
// 64 x 64 tile of the whole workgroup, results visible to it after a barrier.
struct GDStep {
    GDiag w;
    GemmArgs s, t, m;
};

__global__ void __launch_bounds__(256) grouped_dstep_kernel(const GDStep* d)
{
#if defined(__HIP_DEVICE_COMPILE__)   // the host pass needs only the launch stub
    __shared__ double lds[TileLds<double, 64, 64, 16>::elems];
    const GDStep* t = d + blockIdx.x;
    {
        // W = tril(Dbar - P): four elements per pass, all their slice loads
        // issued before the (in-order) sums
        const GDiag w = t->w;
        for (int e0 = threadIdx.x; e0 < kGB * kGB; e0 += 4 * 256) {
            double sl[4][kPSlices], d[4];
            bool in[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * 256, r = e / kGB, c = e % kGB;
                in[u] = r < w.kb && c <= r;
                d[u] = in[u] ? w.A[r * w.lda + c] : 0.0;
#pragma unroll
                for (int z = 0; z < kPSlices; ++z) sl[u][z] = in[u] && z < w.np ? w.P[z * kGB * kGB + e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                double p = 0.0;
#pragma unroll
                for (int z = 0; z < kPSlices; ++z)
                    if (z < w.np) p += sl[u][z];   // slices in order
                w.X[e0 + u * 256] = in[u] ? d[u] - p : 0.0;
            }
        }
    }
    __syncthreads();
    {
        const GemmArgs g = t->s;
        gemm_tile<double, 64, 64, 16, 2, 2, true, false, EPI_SYMLOW, false, double>(g, 0, 0, 0, lds);
    }
    __syncthreads();
    {
        const GemmArgs g = t->t;
        gemm_tile<double, 64, 64, 16, 2, 2, false, false, EPI_STORE, false, double>(g, 0, 0, 0, lds);
    }
    __syncthreads();
    {
        const GemmArgs g = t->m;
        gemm_tile<double, 64, 64, 16, 2, 2, true, false, EPI_PHI, false, double>(g, 0, 0, 0, lds);
    }
#endif
}

__global__ void __launch_bounds__(256, 2) grouped_potrf_kernel(const GDiag* d)
{
    __shared__ double F[(kGB / 16) * 256], LU[256];
    const GDiag t = d[blockIdx.x];
    diag_tile_factor_inverse<kGB / 16>(t.kb, t.A, t.lda, t.X, kGB, t.info, t.col0, F, LU);
}

__global__ void __launch_bounds__(256) grouped_inverse_kernel(const GDiag* d)
{
    __shared__ double Ls[kGB * (kGB + 1)];
    __shared__ double rowbuf[kGB];
    const GDiag t = d[blockIdx.x];
    diag_inverse<kGB / 16>(t.kb, t.A, t.lda, t.X, kGB, Ls, rowbuf);
}

__global__ void grouped_info_kernel(int32_t* info, const int32_t* idx, int nb)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < nb) info[idx[i]] = 0;
}

// strict upper triangle of member blockIdx.x := 0; blockIdx.y takes rows
// blockIdx.y, blockIdx.y + gridDim.y, ...
__global__ void __launch_bounds__(256) grouped_zero_kernel(const GZero* z)
{
    const GZero t = z[blockIdx.x];
    for (int64_t r = blockIdx.y; r < t.n; r += gridDim.y)
        for (int64_t c = r + 1 + threadIdx.x; c < t.n; c += 256) t.A[r * t.n + c] = 0.0;
}

enum GOpKind : int {
    G_INFO = 0, G_POTRF, G_INV, G_ZERO,
    G_PANEL_F,      // <double, MK, NK, STORE>            L21 = A21 X^T (in place)
    G_TRAIL,        // <TU, MK, NK, SUB, lower>           A22 -= L21 L21^T (both panels of a step pair)
    G_NARROW,       // <TU, MK, NK, SUB>, C upper masked  next block's columns -= L21 L21^T
    G_PANEL_A,      // <double, MK, KN, STORE>            Cbar = Cbar X (in place)
    G_P_BBAR,       // slices of P = Cbar^T C, and Bbar -= Cbar R (TU), in one launch
    G_DSTEP,        // W, S, T, M of the diagonal step, one workgroup per member
    G_RBAR          // <TU, KM, KN, SUB>                  Rbar -= [M; Cbar]^T [R; B]
};

}  // namespace

// One launch of the schedule: its kind, where its descriptors start in the
// device buffer (bytes), how many workgroups it has.
struct GroupedOp {
    int kind;
    int64_t off;
    int64_t count;
    int64_t off2;   // G_* products: the tile list (the argument array is at off)
    int64_t off3 = 0, off4 = 0, count1 = 0;   // G_P_BBAR: second list's arguments and tiles; first list's count
};

struct GroupedSchedule {
    std::vector<GroupedOp> ops;
    void* dbuf = nullptr;
    double* scratch = nullptr;
    double* invs = nullptr;   // inverses of every 64-block of every member (reverse sweep)
    bool mixed = false;
    hipEvent_t fork = nullptr, join = nullptr;   // the zero-fill branch on a second stream
    size_t fork_op = 0;                          // the branch forks before ops[fork_op]
};

namespace {

// Host-side assembly of the descriptor buffer.
struct Builder {
    std::vector<unsigned char> bytes;
    std::vector<GroupedOp> ops;
    template <typename T>
    int64_t put(const std::vector<T>& v)
    {
        const int64_t off = ((int64_t)bytes.size() + 255) / 256 * 256;
        bytes.resize(off + sizeof(T) * v.size());
        if (!v.empty()) memcpy(bytes.data() + off, v.data(), sizeof(T) * v.size());
        return off;
    }
    void diag(int kind, const std::vector<GDiag>& d)
    {
        if (!d.empty()) ops.push_back({kind, put(d), (int64_t)d.size(), 0});
    }
    void gemm(int kind, const std::vector<GemmArgs>& a, const std::vector<GTile>& t)
    {
        if (t.empty()) return;
        const int64_t oa = put(a);
        ops.push_back({kind, oa, (int64_t)t.size(), put(t)});
    }
    void gemm2(int kind, const std::vector<GemmArgs>& a1, const std::vector<GTile>& t1,
               const std::vector<GemmArgs>& a2, const std::vector<GTile>& t2)
    {
        if (t1.empty() && t2.empty()) return;
        GroupedOp op{kind, put(a1), (int64_t)(t1.size() + t2.size()), put(t1)};
        op.off3 = put(a2);
        op.off4 = put(t2);
        op.count1 = (int64_t)t1.size();
        ops.push_back(op);
    }
};

GemmArgs garg(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
              int64_t ldc)
{
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda;
    g.B = B; g.ldb = ldb;
    g.C = C; g.ldc = ldc;
    g.kchunk = K > 0 ? K : 1;
    return g;
}

void add_tiles(std::vector<GTile>& t, int arg, int64_t M, int64_t N, bool lower)
{
    const int64_t tm = (M + 63) / 64, tn = (N + 63) / 64;
    for (int64_t i = 0; i < tm; ++i)
        for (int64_t j = 0; j < (lower ? i + 1 : tn); ++j) t.push_back({arg, (int32_t)i, (int32_t)j, 0});
}

template <typename TI, bool AKM, bool BNK, int EPI, bool LOWER>
hipError_t launch_gemm(hipStream_t s, const unsigned char* base, const GroupedOp& op)
{
    hipLaunchKernelGGL((grouped_gemm_kernel<TI, AKM, BNK, EPI, LOWER>), dim3((unsigned)op.count), dim3(256), 0, s,
                       (const GemmArgs*)(base + op.off), (const GTile*)(base + op.off2));
    return hipGetLastError();
}

template <typename TU>
hipError_t launch_p_bbar(hipStream_t s, const unsigned char* base, const GroupedOp& op)
{
    hipLaunchKernelGGL(grouped_p_bbar_kernel<TU>, dim3((unsigned)op.count), dim3(256), 0, s,
                       (const GemmArgs*)(base + op.off), (const GTile*)(base + op.off2), (int)op.count1,
                       (const GemmArgs*)(base + op.off3), (const GTile*)(base + op.off4));
    return hipGetLastError();
}

hipError_t launch_dstep(hipStream_t s, const unsigned char* base, const GroupedOp& op)
{
    hipLaunchKernelGGL(grouped_dstep_kernel, dim3((unsigned)op.count), dim3(256), 0, s,
                       (const GDStep*)(base + op.off));
    return hipGetLastError();
}

}  // namespace

int64_t grouped_scratch_doubles(int nb) { return (int64_t)nb * kGScr * kGB * kGB; }

// tasks: members (any order; info index tasks[i].idx, offset tasks[i].off,
// leading dimension n).  mode: 1 factor, 2 reverse sweep, 4 FP32 products.
// Allocates the descriptor buffer and the members' scratch (freed by
// grouped_free) and uploads the descriptors (synchronous copy).
GroupedSchedule* grouped_prepare(int nb, const BatchTask* tasks, double* Abase, double* Lbbase, int32_t* info,
                                 int mode, hipError_t* err)
{
    GroupedSchedule* gp = new GroupedSchedule();
    GroupedSchedule& g = *gp;
    g.mixed = (mode & 4) != 0;
    hipError_t e = hipMalloc((void**)&g.scratch, sizeof(double) * (size_t)std::max<int64_t>(1, grouped_scratch_doubles(nb)));
    if (e != hipSuccess) {
        *err = e;
        grouped_free(gp);
        return nullptr;
    }
    auto scr = [&](int i, int which) { return g.scratch + ((int64_t)i * kGScr + which) * kGB * kGB; };
    Builder B;
    int maxn = 0;
    for (int i = 0; i < nb; ++i) maxn = std::max(maxn, tasks[i].n);
    const int steps = (maxn + kGB - 1) / kGB;
    std::vector<int32_t> idx(nb);
    for (int i = 0; i < nb; ++i) idx[i] = tasks[i].idx;
    const int64_t idx_off = B.put(idx);
    // inverses of every 64-block of every member, for the reverse sweep: the
    // factor's diagonal steps write them when both run in one call, else one
    // launch forms them from L
    std::vector<int64_t> inv0(nb);
    int64_t nblk_all = 0;
    for (int i = 0; i < nb; ++i) {
        inv0[i] = nblk_all;
        nblk_all += (tasks[i].n + kGB - 1) / kGB;
    }
    if (mode & 2) {
        e = hipMalloc((void**)&g.invs, sizeof(double) * (size_t)std::max<int64_t>(1, nblk_all * kGB * kGB));
        if (e != hipSuccess) {
            *err = e;
            grouped_free(gp);
            return nullptr;
        }
    }
    auto invp = [&](int i, int q) { return g.invs + (inv0[i] + q) * kGB * kGB; };
    // the zero fills fork where the factor's last 8 steps begin (their
    // launches are small, so the fills' writes crowd out little), else at
    // the start
    size_t fork_op = 0;
    if (mode & 1) {
        B.ops.push_back({G_INFO, idx_off, nb, 0});
        // Steps in pairs (s even, s + 1): step s updates only block s+1's
        // columns ("narrow"); step s+1 updates the rest with both panels,
        // columns [k - 64, k + 64) of the rows below block s+1, as one
        // product of inner dimension 128.
        for (int s = 0; s < steps; ++s) {
            if (s == std::max(0, steps - 8)) fork_op = B.ops.size();
            std::vector<GDiag> dg;
            std::vector<GemmArgs> pa, ta, na;
            std::vector<GTile> pt, tt, nt;
            for (int i = 0; i < nb; ++i) {
                const int n = tasks[i].n, k = s * kGB;
                if (k >= n) continue;
                const int kb = std::min(kGB, n - k);
                double* A = Abase + tasks[i].off;
                double* X = (mode & 2) ? invp(i, s) : scr(i, kScrX);
                dg.push_back({A + (int64_t)k * n + k, nullptr, X, info + tasks[i].idx, n, k, kb, 0});
                const int64_t m = n - k - kb;
                if (m <= 0) continue;
                double* A21 = A + (int64_t)(k + kb) * n + k;
                pa.push_back(garg(m, kb, kb, A21, n, X, kGB, A21, n));
                add_tiles(pt, (int)pa.size() - 1, m, kb, false);
                if (s % 2 == 0) {
                    const int64_t nn = std::min<int64_t>(kGB, m);
                    GemmArgs gn = garg(m, nn, kb, A21, n, A21, n, A21 + kb, n);
                    gn.c_lower = 1;
                    na.push_back(gn);
                    add_tiles(nt, (int)na.size() - 1, m, nn, false);
                } else {   // block s-1 is whole and precedes this one
                    ta.push_back(garg(m, m, kGB + kb, A21 - kGB, n, A21 - kGB, n, A21 + kb, n));
                    add_tiles(tt, (int)ta.size() - 1, m, m, true);
                }
            }
            B.diag(G_POTRF, dg);
            B.gemm(G_PANEL_F, pa, pt);
            B.gemm(G_NARROW, na, nt);
            B.gemm(G_TRAIL, ta, tt);
        }
        std::vector<GZero> z;
        for (int i = 0; i < nb; ++i)
            if (tasks[i].n > 1) z.push_back({Abase + tasks[i].off, tasks[i].n});
        if (!z.empty()) B.ops.push_back({G_ZERO, B.put(z), (int64_t)z.size(), 0});
    }
    if (mode & 2) {
        if (!(mode & 1)) {   // inverses of all diagonal blocks of all members, one launch up front
            std::vector<GDiag> inv;
            for (int i = 0; i < nb; ++i) {
                const int n = tasks[i].n;
                const double* L = Abase + tasks[i].off;
                for (int q = 0; q * kGB < n; ++q) {
                    const int j = q * kGB, bq = std::min(kGB, n - j);
                    inv.push_back(
                        {const_cast<double*>(L + (int64_t)j * n + j), nullptr, invp(i, q), nullptr, n, 0, bq, 0});
                }
            }
            B.diag(G_INV, inv);
        }
        for (int s = 0; s < steps; ++s) {
            std::vector<GDStep> ds;
            std::vector<GemmArgs> pa, ba, pp, ra;
            std::vector<GTile> pt, bt, ppt, rt;
            for (int i = 0; i < nb; ++i) {
                const int n = tasks[i].n;
                const int nblk = (n + kGB - 1) / kGB, q = nblk - 1 - s;
                if (q < 0) continue;
                const int j = q * kGB, k = std::min(n, j + kGB), bq = k - j, nr = n - k;
                const double* L = Abase + tasks[i].off;
                double* Lb = Lbbase + tasks[i].off;
                const double* D = L + (int64_t)j * n + j;
                double* Dbar = Lb + (int64_t)j * n + j;
                double* Cbar = Lb + (int64_t)k * n + j;
                double *X = invp(i, q), *P = scr(i, kScrP), *W = scr(i, kScrW), *S = scr(i, kScrS),
                       *T = scr(i, kScrT), *M = scr(i, kScrM);
                // P = Cbar^T C: its inner dimension nr split into slices of at
                // least 128 (at most kPSlices), summed in order by the W step
                const int np = nr > 0 ? (int)std::min<int64_t>(kPSlices, std::max<int64_t>(1, nr / 128)) : 0;
                if (nr > 0) {
                    pa.push_back(garg(nr, bq, bq, Cbar, n, X, kGB, Cbar, n));
                    add_tiles(pt, (int)pa.size() - 1, nr, bq, false);
                    // Bbar -= Cbar R in pairs of the member's steps (q0, q0 - 1),
                    // q0 = nblk-2, nblk-4, ...: step q0 updates only block
                    // q0-1's columns, step q0-1 all columns with both terms
                    // (inner dimension 128, its first row block stopping at 64)
                    const bool ingrp = q >= 1 && q <= nblk - 2;
                    const int top = ingrp ? q + (nblk - 2 - q) % 2 : q;
                    const int terms = ingrp ? top - q + 1 : 1;
                    const bool defer = ingrp && q > std::max(1, top - 1);
                    if (defer) {
                        ba.push_back(garg(nr, kGB, bq, Cbar, n, L + (int64_t)j * n + (j - kGB), n,
                                          Lb + (int64_t)k * n + (j - kGB), n));
                        add_tiles(bt, (int)ba.size() - 1, nr, kGB, false);
                    } else if (j > 0) {
                        GemmArgs gb = garg(nr, j, terms * bq, Cbar, n, L + (int64_t)j * n, n, Lb + (int64_t)k * n, n);
                        if (terms > 1) gb.kstep = kGB;
                        ba.push_back(gb);
                        add_tiles(bt, (int)ba.size() - 1, nr, j, false);
                    }
                    GemmArgs gp = garg(bq, bq, nr, Cbar, n, L + (int64_t)k * n + j, n, P, kGB);
                    gp.kchunk = ((nr + np - 1) / np + 15) / 16 * 16;
                    gp.pstride = kGB * kGB;
                    pp.push_back(gp);
                    for (int z = 0; z * gp.kchunk < nr; ++z) ppt.push_back({(int)pp.size() - 1, 0, 0, z});
                }
                GDStep d{};
                d.w = {Dbar, P, W, nullptr, n, 0, bq, nr > 0 ? (int)((nr + pp.back().kchunk - 1) / pp.back().kchunk) : 0};
                d.s = garg(bq, bq, bq, D, n, W, kGB, S, kGB);
                d.s.a_lower = 1;
                d.t = garg(bq, bq, bq, S, kGB, X, kGB, T, kGB);
                d.m = garg(bq, bq, bq, X, kGB, T, kGB, M, kGB);
                d.m.C2 = Dbar;
                d.m.ldc2 = n;
                ds.push_back(d);
                if (j > 0) {
                    GemmArgs gr = garg(bq, j, bq + nr, Cbar, n, L + (int64_t)j * n, n, Lb + (int64_t)j * n, n);
                    gr.Ahead = M;
                    gr.ldah = kGB;
                    gr.head_k = bq;
                    ra.push_back(gr);
                    add_tiles(rt, (int)ra.size() - 1, bq, j, false);
                }
            }
            B.gemm(G_PANEL_A, pa, pt);
            B.gemm2(G_P_BBAR, pp, ppt, ba, bt);
            if (!ds.empty()) B.ops.push_back({G_DSTEP, B.put(ds), (int64_t)ds.size(), 0});
            B.gemm(G_RBAR, ra, rt);
        }
        std::vector<GZero> z;
        for (int i = 0; i < nb; ++i)
            if (tasks[i].n > 1) z.push_back({Lbbase + tasks[i].off, tasks[i].n});
        if (!z.empty()) B.ops.push_back({G_ZERO, B.put(z), (int64_t)z.size(), 0});
    }
    g.fork_op = fork_op < B.ops.size() ? fork_op : 0;
    e = hipEventCreateWithFlags(&g.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g.join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&g.dbuf, std::max<size_t>(256, B.bytes.size()));
    if (e == hipSuccess) e = hipMemcpy(g.dbuf, B.bytes.data(), B.bytes.size(), hipMemcpyHostToDevice);
    g.ops = std::move(B.ops);
    *err = e;
    if (e != hipSuccess) {
        grouped_free(gp);
        return nullptr;
    }
    return gp;
}

// side: a second stream for the zero fills of the strict upper triangles,
// which no other launch reads or writes, so that they overlap the block steps
// (the branch forks from s before ops[fork_op] and joins it at the end);
// nullptr: all on s.
hipError_t grouped_enqueue(const GroupedSchedule* gp, hipStream_t s, hipStream_t side, int32_t* info)
{
    const GroupedSchedule& g = *gp;
    const unsigned char* base = (const unsigned char*)g.dbuf;
    const bool fork = side && g.fork && g.join;
    for (size_t oi = 0; oi < g.ops.size(); ++oi) {
        const GroupedOp& op = g.ops[oi];
        hipError_t e = hipSuccess;
        if (fork && oi == g.fork_op) {
            e = hipEventRecord(g.fork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(side, g.fork, 0);
            for (const GroupedOp& z : g.ops) {
                if (z.kind != G_ZERO || e != hipSuccess) continue;
                hipLaunchKernelGGL(grouped_zero_kernel, dim3((unsigned)z.count, 16), dim3(256), 0, side,
                                   (const GZero*)(base + z.off));
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipEventRecord(g.join, side);
            if (e != hipSuccess) return e;
        }
        const dim3 grid((unsigned)op.count);
        if (fork && op.kind == G_ZERO) continue;
        switch (op.kind) {
        case G_INFO:
            hipLaunchKernelGGL(grouped_info_kernel, dim3((unsigned)((op.count + 255) / 256)), dim3(256), 0, s, info,
                               (const int32_t*)(base + op.off), (int)op.count);
            e = hipGetLastError();
            break;
        case G_POTRF:
            hipLaunchKernelGGL(grouped_potrf_kernel, grid, dim3(256), 0, s, (const GDiag*)(base + op.off));
            e = hipGetLastError();
            break;
        case G_INV:
            hipLaunchKernelGGL(grouped_inverse_kernel, grid, dim3(256), 0, s, (const GDiag*)(base + op.off));
            e = hipGetLastError();
            break;
        case G_ZERO:
            hipLaunchKernelGGL(grouped_zero_kernel, dim3((unsigned)op.count, 16), dim3(256), 0, s,
                               (const GZero*)(base + op.off));
            e = hipGetLastError();
            break;
        case G_PANEL_F: e = launch_gemm<double, false, true, EPI_STORE, false>(s, base, op); break;
        case G_TRAIL:
            e = g.mixed ? launch_gemm<float, false, true, EPI_SUB, true>(s, base, op)
                        : launch_gemm<double, false, true, EPI_SUB, true>(s, base, op);
            break;
        case G_NARROW:
            e = g.mixed ? launch_gemm<float, false, true, EPI_SUB, false>(s, base, op)
                        : launch_gemm<double, false, true, EPI_SUB, false>(s, base, op);
            break;
        case G_PANEL_A: e = launch_gemm<double, false, false, EPI_STORE, false>(s, base, op); break;
        case G_P_BBAR: e = g.mixed ? launch_p_bbar<float>(s, base, op) : launch_p_bbar<double>(s, base, op); break;
        case G_DSTEP: e = launch_dstep(s, base, op); break;
        case G_RBAR:
            e = g.mixed ? launch_gemm<float, true, false, EPI_SUB, false>(s, base, op)
                        : launch_gemm<double, true, false, EPI_SUB, false>(s, base, op);
            break;
        default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return fork ? hipStreamWaitEvent(s, g.join, 0) : hipSuccess;
}

void grouped_free(GroupedSchedule* g)
{
    if (!g) return;
    if (g->dbuf) (void)hipFree(g->dbuf);
    if (g->scratch) (void)hipFree(g->scratch);
    if (g->invs) (void)hipFree(g->invs);
    if (g->fork) (void)hipEventDestroy(g->fork);
    if (g->join) (void)hipEventDestroy(g->join);
    delete g;
}

}  // namespace gpc
