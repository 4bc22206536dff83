// Many covariance matrices of uneven order, factored and differentiated by
// block steps taken by all members at once ("grouped" schedule of the batched
// entry points).
//
// The persistent kernel (batched.hip) gives each matrix to one workgroup, so
// the largest members set the makespan.  Here every step of the blocked
// algorithms of section 3.3 is one launch over all members that still have
// that step: the diagonal-block factor (one workgroup per member), the panel
// product and the lower-tile trailing update (one workgroup per 64 x 64
// output tile of every member); the reverse sweep likewise (diagonal inverse,
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

constexpr int kGB = 64;   // block size of the grouped schedule
constexpr int kGScr = 6;  // 64 x 64 scratch blocks per member (X, P, W, S, T, M)

struct GTile {
    int32_t arg, tm, tn, pad;
};
struct GDiag {   // factor + inverse of a diagonal block / inverse alone / W = tril(Dbar - P)
    double* A;
    const double* P;   // W step: P (nullptr: none)
    double* X;         // inverse (factor, inverse) / W (W step)
    int32_t* info;
    int64_t lda;
    int64_t col0;
    int32_t kb;
    int32_t pad;
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

// W = tril(Dbar - P) (P absent: tril(Dbar)), kb x kb, leading dimension kGB.
__global__ void __launch_bounds__(256) grouped_wform_kernel(const GDiag* d)
{
    const GDiag t = d[blockIdx.x];
    const int kb = t.kb;
    for (int e = threadIdx.x; e < kGB * kGB; e += 256) {
        const int r = e / kGB, c = e % kGB;
        double v = 0.0;
        if (r < kb && c <= r) v = t.A[r * t.lda + c] - (t.P ? t.P[r * kGB + c] : 0.0);
        t.X[e] = v;
    }
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
    G_INFO = 0, G_POTRF, G_INV, G_WFORM, G_ZERO,
    G_PANEL_F,      // <double, MK, NK, STORE>            L21 = A21 X^T (in place)
    G_TRAIL,        // <TU, MK, NK, SUB, lower>           A22 -= L21 L21^T
    G_PANEL_A,      // <double, MK, KN, STORE>            Cbar = Cbar X (in place); T = S X
    G_BBAR,         // <TU, MK, KN, SUB>                  Bbar -= Cbar R
    G_P,            // <double, KM, KN, STORE>            P = Cbar^T C
    G_S,            // <double, KM, KN, SYMLOW>           S = sym(D^T W)
    G_M,            // <double, KM, KN, PHI>              M = X^T T, Dbar <- Phi(M)
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
};

struct GroupedSchedule {
    std::vector<GroupedOp> ops;
    void* dbuf = nullptr;
    double* scratch = nullptr;
    bool mixed = false;
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
    if (mode & 1) {
        B.ops.push_back({G_INFO, idx_off, nb, 0});
        for (int s = 0; s < steps; ++s) {
            std::vector<GDiag> dg;
            std::vector<GemmArgs> pa, ta;
            std::vector<GTile> pt, tt;
            for (int i = 0; i < nb; ++i) {
                const int n = tasks[i].n, k = s * kGB;
                if (k >= n) continue;
                const int kb = std::min(kGB, n - k);
                double* A = Abase + tasks[i].off;
                dg.push_back({A + (int64_t)k * n + k, nullptr, scr(i, 0), info + tasks[i].idx, n, k, kb, 0});
                const int64_t m = n - k - kb;
                if (m <= 0) continue;
                double* A21 = A + (int64_t)(k + kb) * n + k;
                pa.push_back(garg(m, kb, kb, A21, n, scr(i, 0), kGB, A21, n));
                add_tiles(pt, (int)pa.size() - 1, m, kb, false);
                ta.push_back(garg(m, m, kb, A21, n, A21, n, A21 + kb, n));
                add_tiles(tt, (int)ta.size() - 1, m, m, true);
            }
            B.diag(G_POTRF, dg);
            B.gemm(G_PANEL_F, pa, pt);
            B.gemm(G_TRAIL, ta, tt);
        }
        std::vector<GZero> z;
        for (int i = 0; i < nb; ++i)
            if (tasks[i].n > 1) z.push_back({Abase + tasks[i].off, tasks[i].n});
        if (!z.empty()) B.ops.push_back({G_ZERO, B.put(z), (int64_t)z.size(), 0});
    }
    if (mode & 2) {
        for (int s = 0; s < steps; ++s) {
            std::vector<GDiag> inv, wf;
            std::vector<GemmArgs> pa, ba, pp, sa, tx, ma, ra;
            std::vector<GTile> pt, bt, ppt, st, txt, mt, rt;
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
                double *X = scr(i, 0), *P = scr(i, 1), *W = scr(i, 2), *S = scr(i, 3), *T = scr(i, 4),
                       *M = scr(i, 5);
                inv.push_back({const_cast<double*>(D), nullptr, X, nullptr, n, 0, bq, 0});
                if (nr > 0) {
                    pa.push_back(garg(nr, bq, bq, Cbar, n, X, kGB, Cbar, n));
                    add_tiles(pt, (int)pa.size() - 1, nr, bq, false);
                    if (j > 0) {
                        ba.push_back(garg(nr, j, bq, Cbar, n, L + (int64_t)j * n, n, Lb + (int64_t)k * n, n));
                        add_tiles(bt, (int)ba.size() - 1, nr, j, false);
                    }
                    pp.push_back(garg(bq, bq, nr, Cbar, n, L + (int64_t)k * n + j, n, P, kGB));
                    add_tiles(ppt, (int)pp.size() - 1, bq, bq, false);
                }
                wf.push_back({Dbar, nr > 0 ? P : nullptr, W, nullptr, n, 0, bq, 0});
                GemmArgs gs = garg(bq, bq, bq, D, n, W, kGB, S, kGB);
                gs.a_lower = 1;
                sa.push_back(gs);
                add_tiles(st, (int)sa.size() - 1, bq, bq, false);
                tx.push_back(garg(bq, bq, bq, S, kGB, X, kGB, T, kGB));
                add_tiles(txt, (int)tx.size() - 1, bq, bq, false);
                GemmArgs gm = garg(bq, bq, bq, X, kGB, T, kGB, M, kGB);
                gm.C2 = Dbar;
                gm.ldc2 = n;
                ma.push_back(gm);
                add_tiles(mt, (int)ma.size() - 1, bq, bq, false);
                if (j > 0) {
                    GemmArgs gr = garg(bq, j, bq + nr, Cbar, n, L + (int64_t)j * n, n, Lb + (int64_t)j * n, n);
                    gr.Ahead = M;
                    gr.ldah = kGB;
                    gr.head_k = bq;
                    ra.push_back(gr);
                    add_tiles(rt, (int)ra.size() - 1, bq, j, false);
                }
            }
            B.diag(G_INV, inv);
            B.gemm(G_PANEL_A, pa, pt);
            B.gemm(G_BBAR, ba, bt);
            B.gemm(G_P, pp, ppt);
            B.diag(G_WFORM, wf);
            B.gemm(G_S, sa, st);
            B.gemm(G_PANEL_A, tx, txt);
            B.gemm(G_M, ma, mt);
            B.gemm(G_RBAR, ra, rt);
        }
        std::vector<GZero> z;
        for (int i = 0; i < nb; ++i)
            if (tasks[i].n > 1) z.push_back({Lbbase + tasks[i].off, tasks[i].n});
        if (!z.empty()) B.ops.push_back({G_ZERO, B.put(z), (int64_t)z.size(), 0});
    }
    e = hipMalloc(&g.dbuf, std::max<size_t>(256, B.bytes.size()));
    if (e == hipSuccess) e = hipMemcpy(g.dbuf, B.bytes.data(), B.bytes.size(), hipMemcpyHostToDevice);
    g.ops = std::move(B.ops);
    *err = e;
    if (e != hipSuccess) {
        grouped_free(gp);
        return nullptr;
    }
    return gp;
}

hipError_t grouped_enqueue(const GroupedSchedule* gp, hipStream_t s, int32_t* info)
{
    const GroupedSchedule& g = *gp;
    const unsigned char* base = (const unsigned char*)g.dbuf;
    for (const GroupedOp& op : g.ops) {
        hipError_t e = hipSuccess;
        const dim3 grid((unsigned)op.count);
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
        case G_WFORM:
            hipLaunchKernelGGL(grouped_wform_kernel, grid, dim3(256), 0, s, (const GDiag*)(base + op.off));
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
        case G_PANEL_A: e = launch_gemm<double, false, false, EPI_STORE, false>(s, base, op); break;
        case G_BBAR:
            e = g.mixed ? launch_gemm<float, false, false, EPI_SUB, false>(s, base, op)
                        : launch_gemm<double, false, false, EPI_SUB, false>(s, base, op);
            break;
        case G_P: e = launch_gemm<double, true, false, EPI_STORE, false>(s, base, op); break;
        case G_S: e = launch_gemm<double, true, false, EPI_SYMLOW, false>(s, base, op); break;
        case G_M: e = launch_gemm<double, true, false, EPI_PHI, false>(s, base, op); break;
        case G_RBAR:
            e = g.mixed ? launch_gemm<float, true, false, EPI_SUB, false>(s, base, op)
                        : launch_gemm<double, true, false, EPI_SUB, false>(s, base, op);
            break;
        default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void grouped_free(GroupedSchedule* g)
{
    if (!g) return;
    if (g->dbuf) (void)hipFree(g->dbuf);
    if (g->scratch) (void)hipFree(g->scratch);
    delete g;
}

}  // namespace gpc
