// Triangular solves with the factor and the log-determinant (the pieces a GP
// log-density needs: z = L^-1 y, alpha = L^-T z, log|K| = 2 sum log L_ii).
//
// The solves sweep the b x b diagonal blocks of L (section 3.2 solves A x = b
// through the inverse of the triangle; here only the diagonal blocks are
// inverted, and the off-diagonal blocks are applied as matrix-vector
// updates).  Several right-hand sides: one launch per block step q, with
// lookahead (below); one right-hand side: the whole sweep in one launch whose
// workgroups hand the blocks' solutions to each other (see the one-launch
// sweeps further down).  Lookahead: with the coupling
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

// Forward sweep, launch q (q = -1: z_0 only).  Workgroups < BS/16 form the
// next block's z; the rest update the rows below the next block with z_q.
template <int BS>
__global__ void __launch_bounds__(256)
trsv_fwd(int64_t n, int nr, int64_t q, const double* L, int64_t ldl, const double* Dinv, const double* Cf,
         double* Y, int64_t ldy, const double* zcur, double* znext, double* B, int64_t ldb)
{
    constexpr int kLook = BS / 16;
    const int64_t jn = (q + 1) * BS;                      // next block
    const int bn = (int)min((int64_t)BS, n - jn);
    const int bc = q >= 0 ? BS : 0;                       // block q is full whenever a next block exists
    if (blockIdx.x < kLook) {
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
template <int BS>
__global__ void __launch_bounds__(256)
trsv_bwd(int64_t n, int nr, int64_t q, int64_t nblk, const double* L, int64_t ldl, const double* Dinv,
         const double* Cb, double* Y, int64_t ldy, const double* xcur, double* xnext, double* B, int64_t ldb)
{
    constexpr int kLook = BS / 16;
    const int64_t jp = (q - 1) * BS;                      // previous block
    const int bp = (int)min((int64_t)BS, n - jp);
    const int bc = q < nblk ? (int)min((int64_t)BS, n - q * BS) : 0;
    if (blockIdx.x < kLook) {
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
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += 8 * 256) {   // eight loads in flight, sums in order
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = i0 + 256 * k;
            v[k] = i < n ? L[i * ldl + i] : 1.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (i0 + 256 * k < n) s += log(v[k]);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = 2.0 * red[0];
}

// ---- one-launch sweeps, one right-hand side --------------------------------
// The work of a sweep is cut into items handed out by a ticket counter in a
// fixed order, one step at a time (forward: block q = 0, 1, ...; transposed:
// q = nblk-1, nblk-2, ...), each step being the strips of block q and then
// its chain items:
//  - a strip item takes SR = 8192/BS rows (forward) or columns (transposed)
//    of block q and forms y'_r = y_r - sum_p L_rp z_p (transposed: the L^T
//    terms) over the blocks p two or more steps before q, one block at a time
//    as each z_p is complete, then writes y' to the workspace;
//  - a chain item forms 16 rows of the block's solution from y' and the
//    solution of the step before through its coupling block (the lookahead
//    formula of the launch-per-block sweep above).
// An item only waits for items with smaller tickets and a ticket is only
// taken by a running workgroup, so the sweep finishes whatever number of its
// workgroups are resident.
//
// Hand-over.  y' and the solution are written to workspace vectors that
// start filled with a signalling NaN, a value arithmetic never produces.
// Every value one workgroup reads from another is read from such a vector
// with device-scope loads until it is no longer that value, so each read is
// its own signal: no read relies on the order in which two different
// locations become visible, and no cache maintenance (L2 write-back or
// invalidate) is needed (device-scope accesses are coherent across the
// per-XCD L2 caches, and no plain load leaves a copy of such data in an L2).
// Per-step counters (one word per workgroup), raised by the chain items once
// their stores have completed, only throttle the polling: a chain item of
// step q waits on the counter of step q-2 before it polls its operands, and
// a strip waits on the counter of each block but its last before it reads
// that block's solution (still checking every value).  So only the few items
// near the front of the sweep poll data, the rest poll one word each.
//
// Every wait is bounded in time (kWaitTicks of the 100 MHz constant clock):
// a wait that runs out raises the sweep's error flag and the caller's
// failure record; later waits then return at once and the chain items write
// NaN, so a sweep that could not finish ends promptly, shows in its result
// and is reported to the host (the library reads the record).  The reduction
// orders are fixed, so results repeat bit for bit.

constexpr uint64_t kWaitTicks = 10000000ull;           // 100 ms at 100 MHz
constexpr int kCtrlStride = 32;                        // words between two counters (128 B)
constexpr uint64_t kPending = 0x7FF0DEADBEEF0001ull;   // signalling NaN: not yet written

// control words: [0] ticket, [kCtrlStride] error flag, then the counters of
// the nblk steps
__host__ __device__ constexpr int64_t ctrl_words(int64_t nblk) { return kCtrlStride * (nblk + 2); }
__device__ __forceinline__ uint32_t* zdone(uint32_t* ctrl, int64_t q) { return ctrl + kCtrlStride * (2 + q); }

__device__ __forceinline__ uint32_t load_agent(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The sweep's shared words: its error flag (reset by every sweep) and the
// caller's failure record (kept across sweeps until the host clears it).
struct SweepFlags {
    uint32_t* err;
    uint32_t* rec;
};

__device__ __forceinline__ void raise_failure(const SweepFlags& f)
{
    store_agent(f.err, 1u);
    store_agent(f.rec, 1u);
}

// True if the sweep has failed; then the caller's record is (also) raised,
// so that a sweep started with its flag raised is reported as well.
__device__ __forceinline__ bool failed(const SweepFlags& f)
{
    if (!load_agent(f.err)) return false;
    store_agent(f.rec, 1u);
    return true;
}

__device__ __forceinline__ uint64_t now_ticks() { return (uint64_t)wall_clock64(); }

// Bounded wait of one thread: true while it may go on polling.  The clock is
// read every 16 polls (the first reading sets the deadline); past the
// deadline the flags are raised, and a raised flag ends every wait.
__device__ __forceinline__ bool keep_polling(uint32_t& it, uint64_t& deadline, const SweepFlags& f)
{
    if ((++it & 15u) == 0) {
        if (load_agent(f.err)) return false;
        const uint64_t t = now_ticks();
        if (deadline == 0) {
            deadline = t + kWaitTicks;
        } else if (t > deadline) {
            raise_failure(f);
            return false;
        }
    }
    __builtin_amdgcn_s_sleep(1);
    return true;
}

// One thread: *p once it is no longer kPending (or the sweep has failed).
// Two reads are kept in flight, the older one checked while the newer is on
// its way, so a value is seen about half a round trip sooner than with one.
__device__ double await_value(const double* p, const SweepFlags& f)
{
    uint32_t it = 0;
    uint64_t deadline = 0;
    double a = ld_dev(p);
    double b = ld_dev(p);
    for (;;) {
        if (__builtin_bit_cast(uint64_t, a) != kPending || !keep_polling(it, deadline, f)) return a;
        a = ld_dev(p);
        if (__builtin_bit_cast(uint64_t, b) != kPending || !keep_polling(it, deadline, f)) return b;
        b = ld_dev(p);
    }
}

// The counter work is done by the whole first wave, with values made uniform
// by readfirstlane, so no branch around a barrier depends on the lane: a
// branch on threadIdx.x == 0 at the end of the item loop lets the compiler
// split the loop in two around it, thread 0 leaving the other lanes (still
// cycling through the barriers) for the counter updates.
__device__ __forceinline__ bool first_wave() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0; }

// All threads: returns once *ctr >= target, or the sweep has failed, or the
// wait ran out of time (then the flags are raised).
__device__ void wait_count(const uint32_t* ctr, uint32_t target, const SweepFlags& f)
{
    if (first_wave()) {
        uint32_t it = 0;
        uint64_t deadline = 0;
        while (__builtin_amdgcn_readfirstlane(load_agent(ctr)) < target) {
            if ((++it & 15u) == 0) {
                if (__builtin_amdgcn_readfirstlane(load_agent(f.err))) break;
                const uint64_t t = now_ticks();   // a scalar read: uniform
                if (deadline == 0) {
                    deadline = t + kWaitTicks;
                } else if (t > deadline) {
                    raise_failure(f);
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
}

// All threads: waits for this workgroup's stores to complete, then adds one
// to *ctr (lane 0 of the first wave adds 1, its other lanes 0).
__device__ void publish(uint32_t* ctr)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (first_wave())
        __hip_atomic_fetch_add(ctr, threadIdx.x == 0 ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Next item of this workgroup (all threads; uniform result).
__device__ uint32_t next_ticket(uint32_t* ctrl)
{
    __shared__ uint32_t s_ticket;
    if (first_wave()) {
        const uint32_t v = __hip_atomic_fetch_add(ctrl, threadIdx.x == 0 ? 1u : 0u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        s_ticket = __builtin_amdgcn_readfirstlane(v);     // lane 0 holds the value before its add
    }
    __syncthreads();
    const uint32_t t = __builtin_amdgcn_readfirstlane(s_ticket);
    __syncthreads();
    return t;
}

// Forward strip: rows [q BS + r SR, +SR) of block q (SR = 8192/BS).  Thread
// (row group g = tid/32, slot s = tid%32) covers rows g, g+8, ... of the strip
// and columns s, s+32, ... of each block p, so that a wave load reads two
// 256-byte row segments; each row's 32 slot sums run over p in increasing
// order and are combined in a fixed tree.
template <int BS>
__device__ void fwd_strip(int64_t n, int64_t q, int r, const double* L, int64_t ldl, const double* B, int64_t ldb,
                          const double* Zs, double* Yp, uint32_t* ctrl, const SweepFlags& f, double* zs)
{
    constexpr int SR = 8192 / BS, RPT = SR / 8, CPT = BS / 32, K = BS / 16;
    static_assert(RPT * CPT == 32, "32 values of L per thread and block");
    const int slot = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int64_t row0 = q * BS + (int64_t)r * SR + g;
    // y is only overwritten (by the solution) after this strip's y' is read,
    // so it is loaded first, off the path of the last block
    double yv[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t row = row0 + 8 * i;
        yv[i] = (slot == 0 && row < n) ? ld_dev(B + row * ldb) : 0.0;
    }
    double acc[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) acc[i] = 0.0;
    for (int64_t p = 0; p + 2 <= q; ++p) {
        double v[RPT][CPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int64_t row = row0 + 8 * i;
            const double* lr = L + (row < n ? row : 0) * ldl + p * BS + slot;
#pragma unroll
            for (int c = 0; c < CPT; ++c) v[i][c] = row < n ? lr[32 * c] : 0.0;
        }
        // all blocks but the last: throttled by the step counter first; the
        // last is on the chain's path and is read as it lands
        if (p + 2 < q) wait_count(zdone(ctrl, p), K, f);
        if ((int)threadIdx.x < BS) zs[threadIdx.x] = await_value(Zs + p * BS + threadIdx.x, f);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int c = 0; c < CPT; ++c) acc[i] += v[i][c] * zs[slot + 32 * c];
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
#pragma unroll
        for (int w = 1; w < 32; w <<= 1) {
            const double o = __shfl_xor(acc[i], w, 64);
            acc[i] = (slot & w) ? o + acc[i] : acc[i] + o;
        }
        const int64_t row = row0 + 8 * i;
        if (slot == 0 && row < n) st_dev(Yp + row, yv[i] - acc[i]);
    }
}

// Forward chain item c of block q: rows [16c, 16c+16) of
// z_q = Dinv_q y'_q - Cf_q z_{q-1}, written to B and Zs.  16 threads per
// row, slot s covering columns s, s+16, ...; the rows of Dinv_q and Cf_q are
// loaded before the waits.
template <int BS>
__device__ void fwd_chain(int64_t n, int64_t q, int c, const double* Dinv, const double* Cf, double* B,
                          int64_t ldb, double* Zs, const double* Yp, uint32_t* ctrl, const SweepFlags& f, double* ys,
                          double* zs)
{
    const int bq = (int)min((int64_t)BS, n - q * BS);
    const int sl = threadIdx.x & 15;
    const int i = 16 * c + (int)(threadIdx.x >> 4);
    const double* Dn = Dinv + q * BS * BS;
    const double* Cn = Cf + q * BS * BS;
    double dv[BS / 16], cv[BS / 16];
#pragma unroll
    for (int m = 0; m < BS / 16; ++m) {
        const int k = sl + 16 * m;
        dv[m] = (i < bq && k <= i) ? Dn[(int64_t)i * BS + k] : 0.0;   // Dinv is lower
        cv[m] = (q >= 1 && i < bq) ? Cn[(int64_t)i * BS + k] : 0.0;
    }
    // until step q-2 is complete y'_q is far off: wait on its counter (one
    // word per workgroup) before reading the data itself
    if (q >= 2) wait_count(zdone(ctrl, q - 2), BS / 16, f);
    if ((int)threadIdx.x < BS)
        ys[threadIdx.x] = (int)threadIdx.x < bq ? await_value(Yp + q * BS + threadIdx.x, f) : 0.0;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int m = 0; m < BS / 16; ++m) t += dv[m] * ys[sl + 16 * m];
    if (q >= 1) {
        if ((int)threadIdx.x < BS) zs[threadIdx.x] = await_value(Zs + (q - 1) * BS + threadIdx.x, f);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < BS / 16; ++m) t -= cv[m] * zs[sl + 16 * m];
    }
#pragma unroll
    for (int w = 1; w < 16; w <<= 1) {
        const double o = __shfl_xor(t, w, 64);
        t = (sl & w) ? o + t : t + o;
    }
    if (sl == 0 && i < bq) {
        const double z = failed(f) ? __builtin_nan("") : t;
        st_dev(Zs + q * BS + i, z);
        B[(q * BS + i) * ldb] = z;
    }
    publish(zdone(ctrl, q));
}

// Transposed strip: columns [q BS + r SR, +SR) of block q.  Thread (group g,
// column j) covers rows g, g + 256/SR, ... of each block p below; the group
// sums run over p in decreasing order and are combined in group order.
template <int BS>
__device__ void bwd_strip(int64_t n, int64_t nblk, int64_t q, int r, const double* L, int64_t ldl, const double* B,
                          int64_t ldb, const double* Zs, double* Yp, uint32_t* ctrl, const SweepFlags& f, double* xs,
                          double* red)
{
    constexpr int SR = 8192 / BS, NG = 256 / SR, K = BS / 16;
    const int j = threadIdx.x % SR, g = threadIdx.x / SR;
    const int64_t col = q * BS + (int64_t)r * SR + j;
    const bool live = col < n;
    const double yv = (g == 0 && live) ? ld_dev(B + col * ldb) : 0.0;   // as in the forward strip
    double acc = 0.0;
    for (int64_t p = nblk - 1; p >= q + 2; --p) {
        const int bp = (int)min((int64_t)BS, n - p * BS);
        double v[32];
        const double* lc = L + (p * BS + g) * ldl + (live ? col : 0);
#pragma unroll
        for (int k = 0; k < 32; ++k) v[k] = (live && g + NG * k < bp) ? lc[(int64_t)NG * k * ldl] : 0.0;
        if (p > q + 2) wait_count(zdone(ctrl, p), K, f);   // as in the forward strip
        if ((int)threadIdx.x < BS)
            xs[threadIdx.x] = (int)threadIdx.x < bp ? await_value(Zs + p * BS + threadIdx.x, f) : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 32; ++k) acc += v[k] * xs[g + NG * k];
        __syncthreads();
    }
    red[threadIdx.x] = acc;                       // red[g * SR + j]
    __syncthreads();
    if (g == 0 && live) {
        double sum = 0.0;
#pragma unroll
        for (int gg = 0; gg < NG; ++gg) sum += red[gg * SR + j];
        st_dev(Yp + col, yv - sum);
    }
}

// Transposed chain item c of block q: rows [16c, 16c+16) of
// x_q = Dinv_q^T y'_q - Cb_q^T x_{q+1}, written to B and Zs.  Thread
// (t-slot g, row 16c + l) covers t = g, g+16, ...; the columns of Dinv_q and
// Cb_q are loaded before the waits; the 16 t-slot sums are combined in slot
// order.
template <int BS>
__device__ void bwd_chain(int64_t n, int64_t nblk, int64_t q, int c, const double* Dinv, const double* Cb, double* B,
                          int64_t ldb, double* Zs, const double* Yp, uint32_t* ctrl, const SweepFlags& f, double* ys,
                          double* xs, double* red)
{
    const int bq = (int)min((int64_t)BS, n - q * BS);
    const int bc = q + 1 < nblk ? (int)min((int64_t)BS, n - (q + 1) * BS) : 0;
    const int l = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int i = 16 * c + l;
    const double* Dp = Dinv + q * BS * BS;
    const double* Cp = Cb + q * BS * BS;
    double dv[BS / 16], cv[BS / 16];
#pragma unroll
    for (int m = 0; m < BS / 16; ++m) {
        const int t = g + 16 * m;
        dv[m] = (i < bq && t >= i && t < bq) ? Dp[(int64_t)t * BS + i] : 0.0;   // (Dinv^T)[i][t], Dinv lower
        cv[m] = (i < bq && t < bc) ? Cp[(int64_t)t * BS + i] : 0.0;
    }
    if (q + 2 < nblk) wait_count(zdone(ctrl, q + 2), BS / 16, f);   // as in the forward chain
    if ((int)threadIdx.x < BS)
        ys[threadIdx.x] = (int)threadIdx.x < bq ? await_value(Yp + q * BS + threadIdx.x, f) : 0.0;
    __syncthreads();
    double part = 0.0;
#pragma unroll
    for (int m = 0; m < BS / 16; ++m) part += dv[m] * ys[g + 16 * m];
    if (bc > 0) {
        if ((int)threadIdx.x < BS)
            xs[threadIdx.x] = (int)threadIdx.x < bc ? await_value(Zs + (q + 1) * BS + threadIdx.x, f) : 0.0;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < BS / 16; ++m) part -= cv[m] * xs[g + 16 * m];
    }
    red[threadIdx.x] = part;                      // red[g * 16 + l]
    __syncthreads();
    if (threadIdx.x < 16 && 16 * c + (int)threadIdx.x < bq) {
        double v = 0.0;
        for (int gg = 0; gg < 16; ++gg) v += red[gg * 16 + threadIdx.x];
        const double x = failed(f) ? __builtin_nan("") : v;
        st_dev(Zs + q * BS + 16 * c + threadIdx.x, x);
        B[(q * BS + 16 * c + threadIdx.x) * ldb] = x;
    }
    publish(zdone(ctrl, q));
}

// One launch of a whole sweep (trans 0: B <- L^-1 B, 1: B <- L^-T B) for one
// right-hand side.  Yp, Zs: n doubles each, filled with kPending; ctrl:
// ctrl_words(nblk) zeroed words; rec: the caller's failure record.
template <int BS, int TRANS>
__global__ void __launch_bounds__(256, 4)
trsv_sweep1(int64_t n, int64_t nblk, const double* L, int64_t ldl, const double* Dinv, const double* Cpl,
            double* B, int64_t ldb, double* Yp, double* Zs, uint32_t* ctrl, uint32_t* rec)
{
    constexpr int NS = BS * BS / 8192, K = BS / 16, P = NS + K;
    __shared__ double s_a[BS], s_b[BS], s_red[256];
    const SweepFlags f{ctrl + kCtrlStride, rec};
    const uint32_t total = (uint32_t)(nblk * P);
    for (;;) {
        const uint32_t t = next_ticket(ctrl);
        if (t >= total) break;
        const int64_t step = t / P;
        const int r = (int)(t % P);
        const int64_t q = TRANS ? nblk - 1 - step : step;
        if (!TRANS) {
            if (r < NS) fwd_strip<BS>(n, q, r, L, ldl, B, ldb, Zs, Yp, ctrl, f, s_a);
            else fwd_chain<BS>(n, q, r - NS, Dinv, Cpl, B, ldb, Zs, Yp, ctrl, f, s_a, s_b);
        } else {
            if (r < NS) bwd_strip<BS>(n, nblk, q, r, L, ldl, B, ldb, Zs, Yp, ctrl, f, s_a, s_red);
            else bwd_chain<BS>(n, nblk, q, r - NS, Dinv, Cpl, B, ldb, Zs, Yp, ctrl, f, s_a, s_b, s_red);
        }
        // every item's lane-dependent tail joins here, so the loop has one
        // back edge that all lanes take together
        __syncthreads();
    }
}

// Zeroes the control words (the error flag: fail) and fills the 2n
// hand-over entries with kPending.
__global__ void sweep_init(uint32_t* ctrl, int64_t words, double* V, int64_t count, int fail)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < words) ctrl[e] = (e == kCtrlStride && fail) ? 1u : 0u;
    if (e < count) V[e] = __builtin_bit_cast(double, kPending);
}

}  // namespace

// running right-hand sides, two z slots, then the control words of the
// one-launch sweep (sized for the smallest block, 128)
int64_t trsm_workspace(int64_t n)
{
    return (int64_t)kRhsGroup * n + 2 * kSolveMax * kRhsGroup + (ctrl_words((n + 127) / 128) + 1) / 2;
}

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
// One right-hand side: fill the hand-over vectors and control words, then
// one launch of at most four workgroups per compute unit.
template <int BS>
hipError_t sweep1(hipStream_t s, int trans, int64_t n, const double* L, int64_t ldl, const double* Dinv,
                  const double* Cpl, double* B, int64_t ldb, double* Y, int cus, int fail, uint32_t* rec)
{
    constexpr int P = BS * BS / 8192 + BS / 16;
    const int64_t nblk = (n + BS - 1) / BS;
    double* Yp = Y;                                   // y' (n), then the solution (n)
    double* Zs = Y + n;
    uint32_t* ctrl = (uint32_t*)(Y + (int64_t)kRhsGroup * n + 2 * kSolveMax * kRhsGroup);
    const int64_t init = std::max<int64_t>(2 * n, ctrl_words(nblk));
    hipLaunchKernelGGL(sweep_init, dim3((unsigned)((init + 255) / 256)), dim3(256), 0, s, ctrl, ctrl_words(nblk), Yp,
                       2 * n, fail);
    const int64_t grid = std::min<int64_t>(nblk * P, 4 * (int64_t)std::max(cus, 1));
    if (!trans)
        hipLaunchKernelGGL((trsv_sweep1<BS, 0>), dim3((unsigned)grid), dim3(256), 0, s, n, nblk, L, ldl, Dinv, Cpl, B,
                           ldb, Yp, Zs, ctrl, rec);
    else
        hipLaunchKernelGGL((trsv_sweep1<BS, 1>), dim3((unsigned)grid), dim3(256), 0, s, n, nblk, L, ldl, Dinv, Cpl, B,
                           ldb, Yp, Zs, ctrl, rec);
    return hipGetLastError();
}

template <int BS>
hipError_t sweep(hipStream_t s, int trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                 const double* Dinv, const double* Cpl, double* B, int64_t ldb, double* Y, int cus, int fail,
                 uint32_t* rec)
{
    constexpr int kLook = BS / 16;
    const int64_t nblk = (n + BS - 1) / BS;
    double* zb = Y + (int64_t)kRhsGroup * n;            // two z slots
    auto zslot = [&](int64_t q) { return zb + (q & 1) * kSolveMax * kRhsGroup; };
    for (int64_t c0 = 0; c0 < nrhs; c0 += kRhsGroup) {
        const int nr = (int)std::min<int64_t>(kRhsGroup, nrhs - c0);
        double* Bc = B + c0;
        if (nr == 1) {
            const hipError_t e = sweep1<BS>(s, trans, n, L, ldl, Dinv, Cpl, Bc, ldb, Y, cus, fail, rec);
            if (e != hipSuccess) return e;
            continue;
        }
        hipLaunchKernelGGL(copy_cols, dim3((unsigned)((n * nr + 255) / 256)), dim3(256), 0, s, n, nr, Bc, ldb, Y,
                           (int64_t)kRhsGroup);
        if (!trans) {
            for (int64_t q = -1; q + 1 < nblk; ++q) {
                const int64_t jn = (q + 1) * BS;
                const int64_t rest = n - std::min(n, jn + BS);
                const int64_t blocks = kLook + (q >= 0 ? (rest + kRows - 1) / kRows : 0);
                hipLaunchKernelGGL((trsv_fwd<BS>), dim3((unsigned)blocks), dim3(256), 0, s, n, nr, q, L, ldl, Dinv,
                                   Cpl, Y, (int64_t)kRhsGroup, zslot(q), zslot(q + 1), Bc, ldb);
            }
        } else {
            for (int64_t q = nblk; q >= 1; --q) {
                const int64_t jp = (q - 1) * BS;
                const int64_t blocks = kLook + (q < nblk ? (jp + 63) / 64 : 0);
                hipLaunchKernelGGL((trsv_bwd<BS>), dim3((unsigned)blocks), dim3(256), 0, s, n, nr, q, nblk, L, ldl,
                                   Dinv, Cpl, Y, (int64_t)kRhsGroup, zslot(q), zslot(q - 1), Bc, ldb);
            }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

hipError_t trsm_blocked(hipStream_t s, int trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                        const double* Dinv, const double* Cpl, int b, double* B, int64_t ldb, double* Y, int cus,
                        int fail, uint32_t* rec)
{
    if (!rec) return hipErrorInvalidValue;
    if (b == 128) return sweep<128>(s, trans, n, nrhs, L, ldl, Dinv, Cpl, B, ldb, Y, cus, fail, rec);
    if (b == 256) return sweep<256>(s, trans, n, nrhs, L, ldl, Dinv, Cpl, B, ldb, Y, cus, fail, rec);
    return hipErrorInvalidValue;
}

hipError_t logdet(hipStream_t s, int64_t n, const double* L, int64_t ldl, double* out)
{
    hipLaunchKernelGGL(logdet_kernel, dim3(1), dim3(256), 0, s, n, L, ldl, out);
    return hipGetLastError();
}

}  // namespace gpc
