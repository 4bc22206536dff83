// Operations beside the Cholesky path: the lower-triangular inverse and the
// products of the triangular-solve and inverse reverse modes (section 3.2),
// general matrix products with split-K for long inner dimensions and the
// C = A A^T special case (section 3.1), and the Bernoulli-logit GLM
// likelihood with its gradient (section 3.4).
#include <algorithm>

#include "diag.hpp"
#include "internal.hpp"

namespace gpc {
namespace {

// ---- lower-triangular inverse ----------------------------------------------

// Inverse of the kDiagMax-block p = blockIdx.x of L written in place into the
// same block of X (leading dimension ldx); its strict upper part is zeroed.
__global__ void __launch_bounds__(256)
trtri_into_kernel(int64_t n, const double* L, int64_t ldl, double* X, int64_t ldx)
{
    __shared__ double Ls[kDiagMax * (kDiagMax + 1)];
    __shared__ double rowbuf[kDiagMax];
    const int64_t r0 = (int64_t)blockIdx.x * kDiagMax;
    const int kb = (int)min((int64_t)kDiagMax, n - r0);
    diag_inverse<kDiagMax / 16>(kb, L + r0 * ldl + r0, ldl, X + r0 * ldx + r0, ldx, Ls, rowbuf);
}

// ---- fixed-order split-K sums ------------------------------------------------

// C[m][n] = beta C[m][n] + sum_{z<S} P[z][m][n] (z increasing, loads issued
// sixteen at a time), beta 0 or 1.
__global__ void reduce_store_kernel(int64_t M, int64_t N, const double* P, int S, int64_t pstride, double beta,
                                    double* C, int64_t ldc)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * N) return;
    const int64_t m = e / N, c = e % N;
    constexpr int G = 16;
    const double* p = P + e;
    double s = 0.0;
    for (int z = 0; z < S; z += G) {
        double v[G];
#pragma unroll
        for (int k = 0; k < G; ++k) v[k] = z + k < S ? p[(int64_t)(z + k) * pstride] : 0.0;
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (z + k < S) s += v[k];
    }
    double* out = C + m * ldc + c;
    *out = beta == 0.0 ? s : *out + s;
}

// ---- Bernoulli-logit GLM -------------------------------------------------------
//
// Memory-bound: X (n x k, row-major) is read once.  A team of G lanes takes
// one row at a time, lane l holding columns l, l + G, ..., l + (V-1) G in
// registers; the row's linear term is a fixed-order butterfly sum across the
// team, after which every lane knows mu_i and d_i = y_i - s(mu_i) and adds
// X_ic d_i to its column accumulators (the gradient's second matrix-vector
// product, fused: the row is still in registers).  A workgroup owns a
// contiguous block of rows; its teams' sums are combined in team order and
// written as one partial row (lp, dalpha, dbeta[k]); a second kernel adds the
// workgroups' partial rows in order.  Wide rows (k > 64 V_max) take two
// passes: mu and d first, then X^T d by row blocks.

__device__ __forceinline__ double softplus(double t) { return fmax(t, 0.0) + log1p(exp(-fabs(t))); }

struct GlmArgs {
    int64_t n, k;
    const double* X;
    int64_t ldx;
    const int32_t* y;
    const double* alpha;
    const double* beta;
    double* dX;
    int64_t lddx;
    double* part;        // [gridDim.x][k + 2]
    double* d;           // two-pass form: d_i (n doubles)
    int64_t rows_per_wg;
};

// lp_i and d_i of one row from its linear term (all lanes of the team).
__device__ __forceinline__ void glm_row(double mu, int32_t yi, double& lp, double& d)
{
    const double yv = (double)yi;
    lp = -yv * softplus(-mu) - (1.0 - yv) * softplus(mu);
    d = yv - 1.0 / (1.0 + exp(-mu));
}

// Team sum of v over G lanes (butterfly; the lower lane's value always on the
// left, so every lane ends with the same bits).
template <int G>
__device__ __forceinline__ double team_sum(double v, int l)
{
#pragma unroll
    for (int w = 1; w < G; w <<= 1) {
        const double o = __shfl_xor(v, w, 64);
        v = (l & w) ? o + v : v + o;
    }
    return v;
}

// Combine per-team values buf[team][slot] (slots [0, W)) in team order into
// part_row[slot]; all threads.
template <int TEAMS>
__device__ void combine_teams(const double* buf, int W, int64_t stride, double* part_row)
{
    for (int c = threadIdx.x; c < W; c += 256) {
        double s = 0.0;
        for (int t = 0; t < TEAMS; ++t) s += buf[(int64_t)t * stride + c];
        part_row[c] = s;
    }
}

template <int G, int V>
__global__ void __launch_bounds__(256) glm_fused_kernel(GlmArgs a)
{
    constexpr int TEAMS = 256 / G;
    constexpr int KC = G * V;                    // columns covered (>= k)
    __shared__ double s_beta[KC];
    __shared__ double buf[TEAMS * (KC + 2)];     // at most 4 x 2050 doubles
    const int tid = threadIdx.x, team = tid / G, l = tid % G;
    const int k = (int)a.k;
    for (int c = tid; c < KC; c += 256) s_beta[c] = c < k ? a.beta[c] : 0.0;
    __syncthreads();
    const double alpha = *a.alpha;
    double acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0;
    double lps = 0.0, das = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.n, r0 + a.rows_per_wg);
    // the next row of the team is loaded before the current one is used, so
    // one row's loads are always in flight behind the arithmetic
    double xn[V];
    int32_t yn = 0;
    auto load_row = [&](int64_t i) {
        const double* xr = a.X + i * a.ldx;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = l + G * v;
            xn[v] = (i < r1 && c < k) ? xr[c] : 0.0;
        }
        yn = i < r1 ? a.y[i] : 0;
    };
    load_row(r0 + team);
    for (int64_t i = r0 + team; i < r1; i += TEAMS) {
        double x[V];
#pragma unroll
        for (int v = 0; v < V; ++v) x[v] = xn[v];
        const int32_t yi = yn;
        load_row(i + TEAMS);
        double t = 0.0;
#pragma unroll
        for (int v = 0; v < V; ++v) t += x[v] * s_beta[l + G * v];
        t = team_sum<G>(t, l);
        double lp, d;
        glm_row(alpha + t, yi, lp, d);
        lps += lp;
        das += d;
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] += x[v] * d;
        if (a.dX) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int c = l + G * v;
                if (c < k) a.dX[i * a.lddx + c] = d * s_beta[c];
            }
        }
    }
    // per-team row of the workgroup buffer: [lp, dalpha, dbeta[KC]]
    const int64_t stride = KC + 2;
    double* row = buf + (int64_t)team * stride;
    if (l == 0) {
        row[0] = lps;
        row[1] = das;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) row[2 + l + G * v] = acc[v];
    __syncthreads();
    combine_teams<TEAMS>(buf, k + 2, stride, a.part + (int64_t)blockIdx.x * (a.k + 2));
}

// Two-pass form, pass 1: mu, lp, d per row (columns streamed in chunks of
// 64 x 16), d_i written out, dX if asked, per-workgroup lp and dalpha.
__global__ void __launch_bounds__(256) glm_wide_mu_kernel(GlmArgs a)
{
    constexpr int G = 64, V = 16, TEAMS = 4;
    __shared__ double s_ld[TEAMS][2];
    const int tid = threadIdx.x, team = tid / G, l = tid % G;
    const int64_t k = a.k;
    const double alpha = *a.alpha;
    double lps = 0.0, das = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.n, r0 + a.rows_per_wg);
    for (int64_t i = r0 + team; i < r1; i += TEAMS) {
        const double* xr = a.X + i * a.ldx;
        double t = 0.0;
        for (int64_t c0 = 0; c0 < k; c0 += G * V) {
            double x[V], b[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int64_t c = c0 + l + G * v;
                x[v] = c < k ? xr[c] : 0.0;
                b[v] = c < k ? a.beta[c] : 0.0;
            }
#pragma unroll
            for (int v = 0; v < V; ++v) t += x[v] * b[v];
        }
        t = team_sum<G>(t, l);
        double lp, d;
        glm_row(alpha + t, a.y[i], lp, d);
        lps += lp;
        das += d;
        if (l == 0) a.d[i] = d;
        if (a.dX)
            for (int64_t c = l; c < k; c += G) a.dX[i * a.lddx + c] = d * a.beta[c];
    }
    if (l == 0) {
        s_ld[team][0] = lps;
        s_ld[team][1] = das;
    }
    __syncthreads();
    if (tid < 2) {
        double s = 0.0;
        for (int t = 0; t < TEAMS; ++t) s += s_ld[t][tid];
        a.part[(int64_t)blockIdx.x * (k + 2) + tid] = s;
    }
}

// Two-pass form, pass 2: dbeta partials of a row block, columns
// [blockIdx.y * 1024, +1024), four per thread; rows in increasing order.
__global__ void __launch_bounds__(256) glm_wide_xtd_kernel(GlmArgs a)
{
    const int64_t k = a.k;
    const int64_t c0 = (int64_t)blockIdx.y * 1024 + threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.n, r0 + a.rows_per_wg);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = r0; i < r1; ++i) {
        const double di = a.d[i];
        const double* xr = a.X + i * a.ldx;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t c = c0 + 256 * v;
            if (c < k) acc[v] += xr[c] * di;
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t c = c0 + 256 * v;
        if (c < k) a.part[(int64_t)blockIdx.x * (k + 2) + 2 + c] = acc[v];
    }
}

// out[s] = sum over the nwg partial rows of slot s = blockIdx.x (slot 0 ->
// lp, 1 -> dalpha, 2 + c -> dbeta[c]): thread t adds rows t, t + 256, ...
// in order, then a fixed tree over the 256 threads.
__global__ void __launch_bounds__(256) glm_reduce_kernel(int64_t nwg, int64_t k, const double* part, double* lp,
                                                         double* dalpha, double* dbeta)
{
    __shared__ double red[256];
    const int64_t sl = blockIdx.x;
    double s = 0.0;
    for (int64_t w = threadIdx.x; w < nwg; w += 256) s += part[w * (k + 2) + sl];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (sl == 0) *lp = red[0];
        else if (sl == 1) *dalpha = red[0];
        else dbeta[sl - 2] = red[0];
    }
}

template <int G, int V>
hipError_t glm_fused_launch(hipStream_t s, const GlmArgs& a, int64_t nwg)
{
    hipLaunchKernelGGL((glm_fused_kernel<G, V>), dim3((unsigned)nwg), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t trtri_full(hipStream_t s, int64_t n, const double* L, int64_t ldl, double* X, int64_t ldx)
{
    if (n <= 0) return hipSuccess;
    const int64_t nsub = (n + kDiagMax - 1) / kDiagMax;
    hipLaunchKernelGGL(trtri_into_kernel, dim3((unsigned)nsub), dim3(256), 0, s, n, L, ldl, X, ldx);
    hipError_t e = hipGetLastError();
    // Levels of the divide-and-conquer step of section 3.2: with C1, C2 the
    // inverses of two neighbouring diagonal blocks of size w and A3 the block
    // of L below C1 and left of C2, the block of X there is C3 = -C2 A3 C1.
    // T^T = C1^T A3^T is parked in the (unused) strict upper triangle of X
    // at the mirror position of C3, then C3 = -C2 T; the upper triangle is
    // zeroed at the end.  Full pairs of a level run as one batched launch,
    // a ragged last pair as another.
    for (int64_t w = kDiagMax; w < n && e == hipSuccess; w *= 2) {
        const int64_t pair = 2 * w;
        const int64_t full = n / pair;                 // pairs with both halves of width w
        const int64_t rest = n - full * pair;          // rows after them: a ragged pair if > w
        auto level = [&](int64_t p0, int64_t cnt, int64_t w2) -> hipError_t {
            if (cnt <= 0 || w2 <= 0) return hipSuccess;
            const int64_t o = p0 * pair;               // first row/column of pair p0
            GemmArgs t{};                               // T^T (w x w2) = C1^T A3^T
            t.M = w; t.N = w2; t.K = w;
            t.A = X + o * ldx + o; t.lda = ldx;        // C1, read k-major (its transpose)
            t.a_lower = 1;                             // its upper part holds parked blocks
            t.B = L + (o + w) * ldl + o; t.ldb = ldl;  // A3 (w2 x w), read n-major (its transpose)
            t.C = X + o * ldx + o + w; t.ldc = ldx;    // upper mirror block
            t.kchunk = w;
            t.bsA = pair * ldx + pair; t.bsB = pair * ldl + pair; t.bsC = pair * ldx + pair;
            hipError_t r = gemm_f64(s, TILE_128, true, true, EPI_STORE, false, t, 1, (int)cnt);
            if (r != hipSuccess) return r;
            GemmArgs c{};                               // C3 (w2 x w) = -C2 T
            c.M = w2; c.N = w; c.K = w2;
            c.A = X + (o + w) * ldx + o + w; c.lda = ldx;   // C2, lower
            c.a_lower = 1;                                  // (parked blocks above its diagonal)
            c.B = X + o * ldx + o + w; c.ldb = ldx;         // T^T read n-major is T
            c.C = X + (o + w) * ldx + o; c.ldc = ldx;
            c.kchunk = w2;
            c.negate = 1;
            c.bsA = pair * ldx + pair; c.bsB = pair * ldx + pair; c.bsC = pair * ldx + pair;
            return gemm_f64(s, TILE_128, false, true, EPI_STORE, false, c, 1, (int)cnt);
        };
        e = level(0, full, w);
        if (e == hipSuccess && rest > w) e = level(full, 1, rest - w);
    }
    if (e == hipSuccess) e = zero_strict_upper(s, n, X, ldx);
    return e;
}

// Split-K plan (section 3.1, "large k"): the split count s (at most
// max_splits, at least 256 k-values per split, chunk a multiple of 32) that
// minimises the launch's makespan: rounds of `slots` co-resident workgroups
// times the time of one workgroup (its chunk plus, when split, the partial
// slice it writes), plus the fixed-order sum of the s slices.  Costs are in
// units of one k-value of one 128 x 128 tile: a slice write counts 80, its
// sum a third of a unit per tile and split.
void plan_split_k(int64_t tiles, int64_t K, int max_splits, int64_t slots, int* splits, int64_t* chunk)
{
    if (K <= 0) {   // nothing to split (and no chunk to divide by)
        *splits = 1;
        *chunk = 32;
        return;
    }
    int64_t best_s = 1, best_c = std::max<int64_t>(32, (K + 31) / 32 * 32);
    double best = -1.0;
    for (int64_t sp = 1; sp <= max_splits; ++sp) {
        int64_t c = (K + sp - 1) / sp;
        c = (c + 31) / 32 * 32;
        if (sp > 1 && c < 256) break;
        const int64_t se = std::max<int64_t>(1, (K + c - 1) / c);
        if (se != sp) continue;                     // the same plan as a smaller count
        const int64_t rounds = (tiles * se + slots - 1) / slots;
        const double cost = (double)rounds * (double)(c + (se > 1 ? 80 : 0)) + (se > 1 ? 0.32 * tiles * se : 0.0);
        if (best < 0.0 || cost < best) {
            best = cost;
            best_s = se;
            best_c = c;
        }
    }
    *splits = (int)best_s;
    *chunk = best_c;
}

int64_t gemm_general_workspace(int64_t M, int64_t N, int64_t K, int cus, int max_splits)
{
    int sp;
    int64_t ch;
    plan_split_k(((M + 127) / 128) * ((N + 127) / 128), K, max_splits, 2 * (int64_t)cus, &sp, &ch);
    return sp > 1 ? (int64_t)sp * M * N : 0;
}

hipError_t gemm_general(hipStream_t s, bool ta, bool tb, int64_t M, int64_t N, int64_t K, const double* A,
                        int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* ws,
                        int cus, int max_splits, int* splits_out)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    int sp = 1;
    int64_t ch = K;
    if (K > 0) plan_split_k(((M + 127) / 128) * ((N + 127) / 128), K, max_splits, 2 * (int64_t)cus, &sp, &ch);
    if (splits_out) *splits_out = sp;
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda;
    g.B = B; g.ldb = ldb;
    if (sp <= 1 || K == 0) {
        g.C = C; g.ldc = ldc;
        g.kchunk = K > 0 ? K : 1;
        return gemm_f64(s, TILE_128, ta, tb, beta == 0.0 ? EPI_STORE : EPI_ADD, false, g, 1);
    }
    g.C = ws; g.ldc = N;
    g.kchunk = ch;
    g.pstride = M * N;
    hipError_t e = gemm_f64(s, TILE_128, ta, tb, EPI_PARTIAL, false, g, sp);
    if (e != hipSuccess) return e;
    return reduce_store(s, M, N, ws, sp, M * N, beta, C, ldc);
}

hipError_t reduce_store(hipStream_t s, int64_t M, int64_t N, const double* P, int S, int64_t pstride, double beta,
                        double* C, int64_t ldc)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t tot = M * N;
    hipLaunchKernelGGL(reduce_store_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, N, P, S,
                       pstride, beta, C, ldc);
    return hipGetLastError();
}

int64_t glm_workspace(int64_t n, int64_t k)
{
    const int64_t nwg = glm_groups(n, k);
    return nwg * (k + 2) + (k > kGlmFusedMaxK ? n : 0);
}

int64_t glm_groups(int64_t n, int64_t k)
{
    // 2048 workgroups (eight per CU) once there are 16 rows for each, fewer
    // below; the partial rows (nwg x (k + 2) doubles) are then summed by one
    // workgroup per slot
    (void)k;
    return std::max<int64_t>(1, std::min<int64_t>(2048, (n + 15) / 16));
}

hipError_t glm_bernoulli_logit(hipStream_t s, int64_t n, int64_t k, const double* X, int64_t ldx, const int32_t* y,
                               const double* alpha, const double* beta, double* lp, double* dalpha, double* dbeta,
                               double* dX, int64_t lddx, double* ws)
{
    const int64_t nwg = glm_groups(n, k);
    GlmArgs a{};
    a.n = n; a.k = k; a.X = X; a.ldx = ldx; a.y = y; a.alpha = alpha; a.beta = beta;
    a.dX = dX; a.lddx = lddx;
    a.part = ws;
    a.d = ws + nwg * (k + 2);
    a.rows_per_wg = (n + nwg - 1) / nwg;
    hipError_t e = hipSuccess;
    if (k <= kGlmFusedMaxK) {
        // teams of at most 16 lanes up to k = 128 (so that a wave works on
        // four or more rows at once and the per-row likelihood terms are
        // shared by few lanes), wider teams for wider rows
        if (k <= 1) e = glm_fused_launch<1, 1>(s, a, nwg);
        else if (k <= 2) e = glm_fused_launch<2, 1>(s, a, nwg);
        else if (k <= 4) e = glm_fused_launch<4, 1>(s, a, nwg);
        else if (k <= 8) e = glm_fused_launch<8, 1>(s, a, nwg);
        else if (k <= 16) e = glm_fused_launch<16, 1>(s, a, nwg);
        else if (k <= 32) e = glm_fused_launch<16, 2>(s, a, nwg);
        else if (k <= 64) e = glm_fused_launch<16, 4>(s, a, nwg);
        else if (k <= 128) e = glm_fused_launch<16, 8>(s, a, nwg);
        else if (k <= 256) e = glm_fused_launch<32, 8>(s, a, nwg);
        else if (k <= 512) e = glm_fused_launch<32, 16>(s, a, nwg);
        else if (k <= 1024) e = glm_fused_launch<64, 16>(s, a, nwg);
        else e = glm_fused_launch<64, 32>(s, a, nwg);
    } else {
        hipLaunchKernelGGL(glm_wide_mu_kernel, dim3((unsigned)nwg), dim3(256), 0, s, a);
        e = hipGetLastError();
        if (e == hipSuccess) {
            dim3 grid((unsigned)nwg, (unsigned)((k + 1023) / 1024));
            hipLaunchKernelGGL(glm_wide_xtd_kernel, grid, dim3(256), 0, s, a);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(glm_reduce_kernel, dim3((unsigned)(k + 2)), dim3(256), 0, s, nwg, k, ws, lp, dalpha, dbeta);
    return hipGetLastError();
}

}  // namespace gpc
