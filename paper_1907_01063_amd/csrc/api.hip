// C ABI of libgpchol: argument checks, the handle's workspace, and the host
// loops of the blocked algorithms (each step enqueues kernels on the handle's
// stream; nothing here waits for the device except workspace growth).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "gpchol.h"
#include "internal.hpp"

// One traced launch: events around it plus its algorithmic flops and bytes.
struct TraceRec {
    int cls;
    hipEvent_t t0, t1;
    double flops, bytes;
};

// Size buckets of the batched path's tuned inner block.
constexpr int kTuneBuckets = 5;
constexpr int kTuneLimits[kTuneBuckets] = {128, 256, 512, 1024, 1 << 30};   // n < limit

struct BatchPlan {
    int mode = 0;
    const void *A = nullptr, *Lb = nullptr, *info = nullptr;
    std::vector<int32_t> n;
    std::vector<int64_t> off;
    std::vector<int32_t> blocks;   // tuned block per bucket when the plan was made
    gpc::BatchTask* d_tasks = nullptr;
    int32_t* d_counter = nullptr;
    double* d_ws = nullptr;
    int wgs = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double flops = 0.0;
    bool pinned = false;   // recorded into a caller's graph: its buffers must outlive that graph
    int schedule = 1;      // 1 persistent, 2 grouped
    gpc::GroupedSchedule* grouped = nullptr;
};

struct gpc_handle {
    int device = 0;
    int cus = 256;
    int32_t last_splits = 1;             // split count of the last gpc_gemm
    int tune_block[kTuneBuckets] = {64, 64, 64, 64, 64};
    bool tuned = false;
    hipStream_t cap_stream = nullptr;    // private stream used only to capture graphs
    hipStream_t side = nullptr;          // second stream of the lookahead schedules
    std::vector<hipEvent_t> sync_ev;     // ordering events (timing disabled)
    BatchPlan* plan = nullptr;
    hipStream_t stream = nullptr;
    gpc_options opt{};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    double* acopy = nullptr;             // copy of A for the mixed factor's FP64 fallback
    size_t acopy_bytes = 0;
    int32_t fell_back = 0;
    uint32_t* status_dev = nullptr;      // device words: [0] one-launch sweep failure record
    std::vector<BatchPlan*> retired;     // plans a caller's graph may still use (freed at destroy)
    hipEvent_t rebind_ev = nullptr;      // orders a new stream after the old one
    char err[256] = {0};
    bool trace = false;
    std::vector<TraceRec> recs;        // launches recorded since the last reset
    std::vector<hipEvent_t> ev_pool;   // events owned by the handle
    size_t ev_used = 0;
};

// ------------------------------------------------------ no-allocation scratch ---
// Device memory of gpc_factor_noalloc: the inverse of one diagonal block of
// at most kDiagMax x kDiagMax (128 KiB).  Every GPU the library runs on holds
// its own copy until the process ends.  Host code never passes the array's
// name to a kernel: it uses the device address that hipGetSymbolAddress
// returned for the current device (kept in scratch_dev).
static __device__ __align__(256) double scratch[gpc::kDiagMax * gpc::kDiagMax];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `dev`, looked up once per device with that
// device current (nullptr on failure; the HIP error is kept in the handle).
double* scratch_ptr(gpc_handle* h, int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_dev[dev]) return scratch_dev[dev];
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) hipSetDevice(cur);
    if (e != hipSuccess || !p) {
        if (h) snprintf(h->err, sizeof(h->err), "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        return nullptr;
    }
    scratch_dev[dev] = (double*)p;
    return scratch_dev[dev];
}

}  // namespace

namespace {

using namespace gpc;

constexpr int kDefaultBlock = 256;
// Reverse-sweep steps whose Bbar updates are applied together (by default, at most)
constexpr int kDefaultAdjGroup = 2, kMaxAdjGroup = 8;
// Batched calls take the grouped schedule by default once a member is this large.
constexpr int kGroupedMinN = 256;

gpc_status hip_fail(gpc_handle* h, hipError_t e, const char* what)
{
    if (h) snprintf(h->err, sizeof(h->err), "%s: %s", what, hipGetErrorString(e));
    return GPC_ERR_HIP;
}

#define GPC_HIP(h, call)                                        \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return hip_fail((h), e_, #call);  \
    } while (0)

// Grow-only device workspace; waits for the stream before releasing the old one.
gpc_status ensure_ws(gpc_handle* h, size_t bytes)
{
    if (bytes <= h->ws_bytes) return GPC_OK;
    if (h->ws) {
        GPC_HIP(h, hipStreamSynchronize(h->stream));
        GPC_HIP(h, hipFree(h->ws));
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    hipError_t e = hipMalloc(&h->ws, want);
    if (e != hipSuccess) {
        snprintf(h->err, sizeof(h->err), "workspace of %zu bytes: %s", want, hipGetErrorString(e));
        h->ws = nullptr;
        return GPC_ERR_ALLOC;
    }
    h->ws_bytes = want;
    return GPC_OK;
}

hipEvent_t take_event(gpc_handle* h)
{
    if (h->ev_used == h->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->ev_pool.push_back(e);
    }
    return h->ev_pool[h->ev_used++];
}

// Bracket one launch of kernel class `cls` with events when tracing is on.
struct Traced {
    gpc_handle* h;
    TraceRec rec{};
    bool on;
    hipStream_t st;
    Traced(gpc_handle* h_, int cls, double flops, double bytes, hipStream_t s_ = nullptr)
        : h(h_), on(h_->trace), st(s_ ? s_ : h_->stream)
    {
        if (!on) return;
        rec.cls = cls;
        rec.flops = flops;
        rec.bytes = bytes;
        rec.t0 = take_event(h);
        rec.t1 = take_event(h);
        if (!rec.t0 || !rec.t1) { on = false; return; }
        hipEventRecord(rec.t0, st);
    }
    ~Traced()
    {
        if (!on) return;
        hipEventRecord(rec.t1, st);
        h->recs.push_back(rec);
    }
};

void free_plan(BatchPlan* p)
{
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->d_tasks) hipFree(p->d_tasks);
    if (p->d_counter) hipFree(p->d_counter);
    if (p->d_ws) hipFree(p->d_ws);
    gpc::grouped_free(p->grouped);
    delete p;
}

// Drop the handle's current plan: freed now, or at gpc_destroy if a caller's
// graph may still launch with its buffers.
void retire_plan(gpc_handle* h)
{
    BatchPlan* p = h->plan;
    h->plan = nullptr;
    if (!p) return;
    if (p->pinned) h->retired.push_back(p);
    else free_plan(p);
}

int bucket_of(int32_t n)
{
    for (int b = 0; b < kTuneBuckets; ++b)
        if (n < kTuneLimits[b]) return b;
    return kTuneBuckets - 1;
}

// Tuning cache: lines "<arch> <precision> <bucket-limit> <block>".
void load_tune_cache(gpc_handle* h, const char* path)
{
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char arch[64];
    int prec, lim, blk;
    while (fscanf(f, "%63s %d %d %d", arch, &prec, &lim, &blk) == 4) {
        if (strcmp(arch, "gfx950") != 0 || prec != GPC_FP64) continue;
        for (int b = 0; b < kTuneBuckets; ++b)
            if (kTuneLimits[b] == lim && (blk == 32 || blk == 64)) {
                h->tune_block[b] = blk;
                h->tuned = true;
            }
    }
    fclose(f);
}

// i-th ordering event of the current call (grown on demand, reused across calls).
hipEvent_t sync_event(gpc_handle* h, size_t i)
{
    while (h->sync_ev.size() <= i) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        h->sync_ev.push_back(e);
    }
    return h->sync_ev[i];
}

int block_of(const gpc_handle* h) { return h->opt.block > 0 ? h->opt.block : kDefaultBlock; }

// The factor's default outer block: 512 for the FP64 form of large matrices,
// where the trailing update's K of 512 halves its passes over the trailing
// matrix (the diagonal and panel work stays in 128-wide pieces).  The mixed
// form keeps 256: its FP32 sums over K = 512 double the rounding the FP64
// refinement of the solve then has to remove (one more sweep pair).
int factor_block_of(const gpc_handle* h, int64_t n, bool mixed)
{
    if (h->opt.block > 0) return h->opt.block;
    return !mixed && n >= 8192 ? 2 * kDefaultBlock : kDefaultBlock;
}

// Leading dimensions: at least max(1, n) and at most 2^20 elements (the MFMA
// tiles address 128 rows of an operand with 32-bit byte offsets).
constexpr int64_t kMaxLd = int64_t(1) << 20;
bool ld_ok(int64_t n, int64_t ld) { return ld >= std::max<int64_t>(1, n) && ld <= kMaxLd; }

// Byte ranges of two row-major blocks (rows x cols, leading dimension ld)
// intersect.  Empty blocks intersect nothing.
bool overlap(const void* a, int64_t ra, int64_t ca, int64_t lda, const void* b, int64_t rb, int64_t cb, int64_t ldb)
{
    if (!a || !b || ra <= 0 || ca <= 0 || rb <= 0 || cb <= 0) return false;
    const uintptr_t a0 = (uintptr_t)a, a1 = a0 + sizeof(double) * (size_t)((ra - 1) * lda + ca);
    const uintptr_t b0 = (uintptr_t)b, b1 = b0 + sizeof(double) * (size_t)((rb - 1) * ldb + cb);
    return a0 < b1 && b0 < a1;
}

// Split-K plan: the split count s (at most max_splits, at least 256 k-values
// per split, chunk a multiple of 32, the largest BK) that minimises the
// launch's makespan: the number of rounds of `slots` co-resident workgroups
// times the time of one workgroup (its chunk plus the partial slice it
// writes), plus the reduction of the s slices.  Costs are in units of one
// k-value of one 128 x 128 tile; a slice write counts 80 such units and its
// reduction a third of a unit per tile and split.  A launch with a few
// workgroups past a full round takes two rounds, which the plan avoids.
void splitk_plan(int64_t tiles, int64_t K, int max_splits, int64_t slots, int* splits, int64_t* chunk)
{
    if (K <= 0) {   // nothing to split (and no chunk to divide by)
        *splits = 1;
        *chunk = 32;
        return;
    }
    int64_t best_s = 1, best_c = std::max<int64_t>(32, (K + 31) / 32 * 32);
    double best = -1.0;
    for (int64_t s = 1; s <= max_splits; ++s) {
        int64_t c = (K + s - 1) / s;
        c = (c + 31) / 32 * 32;
        if (s > 1 && c < 256) break;
        const int64_t se = std::max<int64_t>(1, (K + c - 1) / c);
        if (se != s) continue;                      // the same plan as a smaller s
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

// Skinny products on the factor's critical path (the narrow updates, whose C
// is disjoint from their operands): 64 x 64 tiles when 128 x 128 tiles would
// leave most of the 2 x 256 workgroup slots empty.
// Block size of the solve sweeps: 256 halves the number of dependent steps
// once the matrix holds a few such blocks.
int solve_block(int64_t n) { return n >= 512 ? 2 * kDiagMax : kDiagMax; }

TileCfg skinny_tile(int64_t M, int64_t N)
{
    const int64_t t128 = ((M + 127) / 128) * ((N + 127) / 128);
    return t128 < 256 ? TILE_64 : TILE_128;
}

// In-place panel products (one tile column spanning all of N <= 128): 64-row
// tiles while 128-row ones would leave CUs without a workgroup.
TileCfg panel_tile(int64_t M, int cus)
{
    return (M + 127) / 128 < 2 * (int64_t)cus ? TILE_64W : TILE_128;
}

GemmArgs gemm_args(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                   int64_t ldb, double* C, int64_t ldc)
{
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda;
    g.B = B; g.ldb = ldb;
    g.C = C; g.ldc = ldc;
    g.kchunk = K > 0 ? K : 1;
    return g;
}

}  // namespace

// b-blocks (b = 256 or 512) from the inverses of their 128-blocks, a level
// at a time: a 2h-block D = [[D1, 0], [D21, D2]] with h-halves has
// D^-1 = [[X1, 0], [-X2 D21 X1, X2]], its corner by two products batched over
// the b-blocks that hold such a 2h-block at the same position (the last,
// ragged b-block's with a shorter second half by two more).
hipError_t gpc::diag_block_inverses(hipStream_t s, int64_t n, int b, const double* L, int64_t ldl, double* Dinv,
                                    double* Tmp)
{
    if (b <= kDiagMax) return trtri_diag_batched(s, n, b, L, ldl, Dinv);
    if (b != 2 * kDiagMax && b != 4 * kDiagMax) return hipErrorInvalidValue;
    const int64_t nblk = (n + b - 1) / b, bb = (int64_t)b * b;
    hipError_t e = fill_f64(s, nblk * bb, Dinv, 0.0);
    if (e == hipSuccess) e = trtri_diag_into(s, n, b, L, ldl, Dinv);
    // the 2h-blocks at position pos of b-blocks q0 .. q0+cnt-1, second half m2 rows
    auto compose = [&](int64_t h, int64_t pos, int64_t q0, int64_t cnt, int64_t m2) -> hipError_t {
        if (cnt <= 0 || m2 <= 0) return hipSuccess;
        const int64_t r0 = q0 * b + pos;
        const double* L21 = L + (r0 + h) * ldl + r0;
        double* X1 = Dinv + q0 * bb + pos * (b + 1);
        double* T0 = Tmp;
        GemmArgs g1 = gemm_args(m2, h, h, L21, ldl, X1, b, T0, h);   // T0 = -D21 X1
        g1.negate = 1;
        g1.bsA = (int64_t)b * ldl + b;
        g1.bsB = bb;
        g1.bsC = h * h;
        hipError_t r = gemm_f64(s, TILE_128, false, false, EPI_STORE, false, g1, 1, (int)cnt);
        if (r != hipSuccess) return r;
        GemmArgs g2 = gemm_args(m2, h, m2, X1 + h * b + h, b, T0, h, X1 + h * b, b);   // X21 = X2 T0
        g2.bsA = bb;
        g2.bsB = h * h;
        g2.bsC = bb;
        return gemm_f64(s, TILE_128, false, false, EPI_STORE, false, g2, 1, (int)cnt);
    };
    for (int64_t h = kDiagMax; h < b && e == hipSuccess; h *= 2) {
        for (int64_t pos = 0; pos < b && e == hipSuccess; pos += 2 * h) {
            // b-blocks whose 2h-block at pos has a whole second half, then the one with a partial one
            const int64_t nfull = n >= pos + 2 * h ? (n - pos - 2 * h) / b + 1 : 0;
            e = compose(h, pos, 0, std::min(nfull, nblk), h);
            if (e == hipSuccess && nfull < nblk) e = compose(h, pos, nfull, 1, n - (nfull * b + pos + h));
        }
    }
    return e;
}

extern "C" {

const char* gpc_status_string(gpc_status s)
{
    switch (s) {
    case GPC_OK: return "ok";
    case GPC_ERR_ARG: return "invalid argument";
    case GPC_ERR_NO_DEVICE: return "no HIP device";
    case GPC_ERR_ARCH: return "device is not gfx950";
    case GPC_ERR_HIP: return "HIP runtime error";
    case GPC_ERR_REFINE: return "iterative refinement did not converge";
    case GPC_ERR_ALLOC: return "workspace allocation failed";
    case GPC_ERR_SWEEP: return "a one-launch solve sweep ran out of time (its results are NaN)";
    case GPC_ERR_CAPTURE: return "the call cannot be recorded into the stream's graph capture as prepared";
    }
    return "unknown status";
}

const char* gpc_last_error(const gpc_handle* h) { return h ? h->err : ""; }

gpc_status gpc_create(gpc_handle** out, void* stream)
{
    if (!out) return GPC_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return GPC_ERR_NO_DEVICE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GPC_ERR_NO_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return GPC_ERR_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GPC_ERR_ARCH;
    gpc_handle* h = new (std::nothrow) gpc_handle();
    if (!h) return GPC_ERR_ALLOC;
    h->device = dev;
    h->stream = (hipStream_t)stream;
    h->opt.precision = GPC_FP64;
    h->opt.block = 0;
    h->opt.lookahead = 1;
    h->opt.refine_maxit = 10;
    h->opt.refine_tol = 1e-12;
    h->opt.mixed_fallback = 0;
    h->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (hipMalloc((void**)&h->status_dev, 256) != hipSuccess || hipMemset(h->status_dev, 0, 256) != hipSuccess ||
        hipEventCreateWithFlags(&h->rebind_ev, hipEventDisableTiming) != hipSuccess) {
        if (h->status_dev) hipFree(h->status_dev);
        delete h;
        return GPC_ERR_HIP;
    }
    load_tune_cache(h, getenv("GPC_TUNE_CACHE"));
    if (!scratch_ptr(h, dev)) {   // the no-allocation entry point's memory on this device
        hipFree(h->status_dev);
        hipEventDestroy(h->rebind_ev);
        delete h;
        return GPC_ERR_HIP;
    }
    *out = h;
    return GPC_OK;
}

gpc_status gpc_destroy(gpc_handle* h)
{
    if (!h) return GPC_ERR_ARG;
    gpc_status st = GPC_OK;
    if (hipStreamSynchronize(h->stream) != hipSuccess) st = GPC_ERR_HIP;
    if (h->ws && hipFree(h->ws) != hipSuccess) st = GPC_ERR_HIP;
    if (h->acopy && hipFree(h->acopy) != hipSuccess) st = GPC_ERR_HIP;
    for (hipEvent_t e : h->ev_pool) hipEventDestroy(e);
    free_plan(h->plan);
    for (BatchPlan* p : h->retired) free_plan(p);
    if (h->status_dev && hipFree(h->status_dev) != hipSuccess) st = GPC_ERR_HIP;
    if (h->rebind_ev) hipEventDestroy(h->rebind_ev);
    if (h->cap_stream) hipStreamDestroy(h->cap_stream);
    if (h->side) hipStreamDestroy(h->side);
    for (hipEvent_t e : h->sync_ev) hipEventDestroy(e);
    delete h;
    return st;
}

gpc_status gpc_trace_enable(gpc_handle* h, int32_t on)
{
    if (!h) return GPC_ERR_ARG;
    h->trace = on != 0;
    return GPC_OK;
}

gpc_status gpc_trace_reset(gpc_handle* h)
{
    if (!h) return GPC_ERR_ARG;
    GPC_HIP(h, hipStreamSynchronize(h->stream));
    h->recs.clear();
    h->ev_used = 0;
    return GPC_OK;
}

gpc_status gpc_trace_read(gpc_handle* h, int32_t kclass, int64_t* launches, double* ms, double* flops,
                          double* bytes)
{
    if (!h || !launches || !ms || !flops || !bytes || kclass < 0 || kclass >= GPC_K_COUNT)
        return GPC_ERR_ARG;
    GPC_HIP(h, hipStreamSynchronize(h->stream));
    *launches = 0;
    *ms = *flops = *bytes = 0.0;
    for (const TraceRec& r : h->recs) {
        if (r.cls != kclass) continue;
        float e = 0.f;
        GPC_HIP(h, hipEventElapsedTime(&e, r.t0, r.t1));
        *launches += 1;
        *ms += e;
        *flops += r.flops;
        *bytes += r.bytes;
    }
    return GPC_OK;
}

gpc_status gpc_set_stream(gpc_handle* h, void* stream)
{
    if (!h) return GPC_ERR_ARG;
    hipStream_t ns = (hipStream_t)stream;
    if (ns == h->stream) return GPC_OK;
    // the handle's workspace may still be in use by work queued on the old
    // stream: the new stream waits for everything enqueued there so far.
    // Not while either stream captures a graph (an event from outside a
    // capture cannot be waited on inside it): a captured graph runs when
    // its caller launches it, ordered by the caller.
    hipStreamCaptureStatus c0 = hipStreamCaptureStatusNone, c1 = hipStreamCaptureStatusNone;
    GPC_HIP(h, hipStreamIsCapturing(h->stream, &c0));
    GPC_HIP(h, hipStreamIsCapturing(ns, &c1));
    if (c0 == hipStreamCaptureStatusNone && c1 == hipStreamCaptureStatusNone) {
        GPC_HIP(h, hipEventRecord(h->rebind_ev, h->stream));
        GPC_HIP(h, hipStreamWaitEvent(ns, h->rebind_ev, 0));
    }
    h->stream = ns;
    return GPC_OK;
}

gpc_status gpc_check(gpc_handle* h)
{
    if (!h) return GPC_ERR_ARG;
    uint32_t rec = 0;
    GPC_HIP(h, hipMemcpyAsync(&rec, h->status_dev, sizeof(rec), hipMemcpyDeviceToHost, h->stream));
    GPC_HIP(h, hipStreamSynchronize(h->stream));
    if (rec == 0) return GPC_OK;
    GPC_HIP(h, fill_i32(h->stream, (int32_t*)h->status_dev, 0));
    return GPC_ERR_SWEEP;
}

gpc_status gpc_set_options(gpc_handle* h, const gpc_options* o)
{
    if (!h || !o) return GPC_ERR_ARG;
    if (o->precision != GPC_FP64 && o->precision != GPC_MIXED) return GPC_ERR_ARG;
    if (o->block != 0 && o->block != 32 && o->block != 64 && o->block != 128 && o->block != 256 &&
        o->block != 512)
        return GPC_ERR_ARG;
    if (o->refine_maxit < 0 || !(o->refine_tol > 0.0)) return GPC_ERR_ARG;
    if (o->mixed_fallback != 0 && o->mixed_fallback != 1) return GPC_ERR_ARG;
    if (o->test_flags != 0 && o->test_flags != 1) return GPC_ERR_ARG;
    if (o->gemm_max_splits < 0 || o->gemm_max_splits > kGemmMaxSplits) return GPC_ERR_ARG;
    if (o->batched_schedule < 0 || o->batched_schedule > 2) return GPC_ERR_ARG;
    if (o->adjoint_group < 0 || o->adjoint_group > kMaxAdjGroup) return GPC_ERR_ARG;
    h->opt = *o;
    return GPC_OK;
}

gpc_status gpc_get_options(const gpc_handle* h, gpc_options* o)
{
    if (!h || !o) return GPC_ERR_ARG;
    *o = h->opt;
    return GPC_OK;
}

// ---------------------------------------------------------------- factor ---
// Right-looking blocked factorisation (section 3.3.1).  Outer block B (256,
// or 512 for the FP64 form of large matrices, by default) for the trailing
// update; within it, 128-wide pieces: factor the diagonal block and form its
// inverse (one workgroup), L21 = A21 inv(L11)^T (MFMA product, in place), and
// update the rest of the outer block's columns with the piece's panel.  The
// trailing update A22 -= P P^T of outer step t is split into the next outer
// block's columns ("narrow", main stream) and the rest ("big", lower tiles
// only).  With lookahead the big update of step t
// runs on a second stream while step t+1's diagonal and panel work proceeds:
//   main: wait big(t-2); panels(t); wait big(t-1); narrow(t); record panel(t)
//   side: wait panel(t); big(t); record big(t)
// (panels(t) touch columns no big(t-1) writes; narrow(t) writes columns
// big(t-1) writes; big(t) needs only panels(t), but starts after narrow(t),
// which the next step's chain waits for; FP32 panel copies of the mixed form
// are double-buffered by step parity, freed by the same waits.)  The strict upper triangle is
// zeroed: with lookahead on the side stream before its first big update,
// else after the last step.
namespace {

// linv_ext: caller-provided room for the diagonal block's inverse (at least
// kDiagMax^2 doubles); the call then allocates nothing: FP64 only, one
// stream, no ordering events, no launch trace.
gpc_status factor_impl(gpc_handle* h, int64_t n, double* A, int64_t lda, int32_t* info, bool mixed,
                       double* linv_ext = nullptr)
{
    hipStream_t s = h->stream;
    GPC_HIP(h, fill_i32(s, info, 0));
    if (n == 0) return GPC_OK;
    const int B = factor_block_of(h, n, mixed);
    const int ib = std::min(B, kDiagMax);
    const size_t n_linv = (size_t)ib * ib;
    const size_t n_pf = mixed ? 2 * (size_t)n * B : 0;
    gpc_status st = GPC_OK;
    double* Linv = linv_ext;
    if (!Linv) {
        st = ensure_ws(h, sizeof(double) * n_linv + sizeof(float) * n_pf);
        if (st != GPC_OK) return st;
        Linv = (double*)h->ws;
    }
    float* Pf2 = (float*)(Linv + n_linv);
    const int64_t steps = (n + B - 1) / B;
    const bool la = !linv_ext && h->opt.lookahead != 0 && steps > 2;
    // with lookahead the main stream's launches (the diagonal chain and the
    // narrow updates) run beside the big update: their waves raise their issue
    // priority, so that a SIMD shared with the big update's waves issues theirs
    // first
    const int cp = la ? 1 : 0;
    hipStream_t s2 = s;
    if (la) {
        if (!h->side) GPC_HIP(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        s2 = h->side;
        hipEvent_t e0 = sync_event(h, 0);
        if (!e0) return GPC_ERR_HIP;
        GPC_HIP(h, hipEventRecord(e0, s));
        GPC_HIP(h, hipStreamWaitEvent(s2, e0, 0));
        // no launch of the factor reads the strict upper triangle, and none
        // writes it but with zeros: clear it here on the side stream, beside
        // the first diagonal steps, not after the last one
        GPC_HIP(h, zero_strict_upper(s2, n, A, lda));
    }
    // events: 1 + 2t = panel and narrow update of step t done, 2 + 2t = big(t)
    auto ev_panel = [&](int64_t t) { return sync_event(h, 1 + 2 * (size_t)t); };
    auto ev_big = [&](int64_t t) { return sync_event(h, 2 + 2 * (size_t)t); };
    if (la && (!ev_panel(steps) || !ev_big(steps))) return GPC_ERR_HIP;

    for (int64_t t = 0; t < steps; ++t) {
        const int64_t k = t * B;
        const int kB = (int)std::min<int64_t>(B, n - k);
        float* Pf = Pf2 + (t & 1) * (size_t)n * B;   // rows k.. of this step's panel, leading dim B
        if (la && t >= 2) GPC_HIP(h, hipStreamWaitEvent(s, ev_big(t - 2), 0));
        for (int h0 = 0; h0 < kB; h0 += ib) {
            const int64_t kh = k + h0;
            const int bh = std::min(ib, kB - h0);
            const double dbh = (double)bh;
            {
                Traced tr(h, GPC_K_DIAG_FACTOR, dbh * dbh * dbh / 3.0, 16.0 * dbh * dbh);
                GPC_HIP(h, potrf_diag(s, bh, A + kh * lda + kh, lda, Linv, ib, info, kh, cp));
            }
            const int64_t m = n - kh - bh;
            if (m <= 0) continue;
            const double dm = (double)m;
            double* P = A + (kh + bh) * lda + kh;
            {
                Traced tr(h, GPC_K_PANEL_SOLVE, dm * dbh * dbh, 8.0 * (2.0 * dm * dbh + dbh * dbh));
                GemmArgs pg = gemm_args(m, bh, bh, P, lda, Linv, ib, P, lda);
                pg.prio = cp;
                if (mixed) {
                    pg.Cf = Pf + (kh + bh - k) * B + h0;
                    pg.ldcf = B;
                }
                // in place: one tile column spans all 128 columns, so no tile writes columns another reads
                GPC_HIP(h, gemm_f64(s, panel_tile(m, h->cus), false, true, EPI_STORE, false, pg, 1));
            }
            if (h0 + bh < kB) {   // the rest of this outer block
                const int nh = kB - h0 - bh;
                const double dnh = (double)nh;
                Traced tr(h, GPC_K_TRAILING_NARROW, 2.0 * dbh * ((dm - dnh) * dnh + dnh * (dnh + 1.0) / 2.0),
                          8.0 * (2.0 * dm * dnh + dm * dbh));
                if (mixed) {
                    const float* Pr = Pf + (kh + bh - k) * B + h0;
                    GemmArgs ng = gemm_args(m, nh, bh, Pr, B, Pr, B, P + bh, lda);
                    ng.c_lower = 1;
                    ng.prio = cp;
                    GPC_HIP(h, gemm_f32in(s, skinny_tile(m, nh), false, true, EPI_SUB, false, ng, 1));
                } else {
                    GemmArgs ng = gemm_args(m, nh, bh, P, lda, P, lda, P + bh, lda);
                    ng.c_lower = 1;
                    ng.prio = cp;
                    GPC_HIP(h, gemm_f64(s, skinny_tile(m, nh), false, true, EPI_SUB, false, ng, 1));
                }
            }
        }
        const int64_t m2 = n - k - kB;
        if (m2 <= 0) break;
        const int64_t nB = std::min<int64_t>(B, m2), mb = m2 - nB;
        const double dkB = (double)kB, dnB = (double)nB, dmb = (double)mb;
        const double* Pd = A + (k + kB) * lda + k;           // panel rows k+kB.., FP64
        const float* Pr = Pf + (size_t)kB * B;               // same rows, FP32 copy
        double* Cn = A + (k + kB) * lda + (k + kB);
        auto big = [&](hipStream_t q) -> gpc_status {
            if (mb <= 0) return GPC_OK;
            Traced tr(h, GPC_K_TRAILING_UPDATE, dmb * (dmb + 1.0) * dkB,
                      (mixed ? 4.0 : 8.0) * dmb * dkB + 8.0 * dmb * (dmb + 1.0), q);
            double* Cb = Cn + nB * lda + nB;
            if (mixed) {
                GemmArgs bg = gemm_args(mb, mb, kB, Pr + nB * B, B, Pr + nB * B, B, Cb, lda);
                GPC_HIP(h, gemm_f32in(q, TILE_128, false, true, EPI_SUB, true, bg, 1));
            } else {
                GemmArgs bg = gemm_args(mb, mb, kB, Pd + nB * lda, lda, Pd + nB * lda, lda, Cb, lda);
                GPC_HIP(h, gemm_f64(q, TILE_128, false, true, EPI_SUB, true, bg, 1));
            }
            return GPC_OK;
        };
        // the next block's columns were last written by big(t-1)
        if (la && t >= 1) GPC_HIP(h, hipStreamWaitEvent(s, ev_big(t - 1), 0));
        {
            Traced tr(h, GPC_K_TRAILING_NARROW, 2.0 * dkB * (dmb * dnB + dnB * (dnB + 1.0) / 2.0),
                      (mixed ? 4.0 : 8.0) * (double)m2 * dkB + 16.0 * (double)m2 * dnB);
            if (mixed) {
                GemmArgs ng = gemm_args(m2, nB, kB, Pr, B, Pr, B, Cn, lda);
                ng.c_lower = 1;
                ng.prio = cp;
                GPC_HIP(h, gemm_f32in(s, skinny_tile(m2, nB), false, true, EPI_SUB, false, ng, 1));
            } else {
                GemmArgs ng = gemm_args(m2, nB, kB, Pd, lda, Pd, lda, Cn, lda);
                ng.c_lower = 1;
                ng.prio = cp;
                GPC_HIP(h, gemm_f64(s, skinny_tile(m2, nB), false, true, EPI_SUB, false, ng, 1));
            }
        }
        if (la) {
            // big(t) needs only this step's panel, but starts after the
            // narrow update: the narrow update, which the next block's chain
            // waits for, then has the CUs to itself, and big(t) runs beside
            // that chain instead
            GPC_HIP(h, hipEventRecord(ev_panel(t), s));
            GPC_HIP(h, hipStreamWaitEvent(s2, ev_panel(t), 0));
            st = big(s2);
            if (st != GPC_OK) return st;
            GPC_HIP(h, hipEventRecord(ev_big(t), s2));
        } else {
            st = big(s);
            if (st != GPC_OK) return st;
        }
    }
    if (la) {   // join the side stream
        hipEvent_t ej = sync_event(h, 0);
        GPC_HIP(h, hipEventRecord(ej, s2));
        GPC_HIP(h, hipStreamWaitEvent(s, ej, 0));
    }
    if (!la) GPC_HIP(h, zero_strict_upper(s, n, A, lda));
    return GPC_OK;
}

}  // namespace

gpc_status gpc_factor(gpc_handle* h, int64_t n, double* A, int64_t lda, int32_t* info)
{
    if (!h || n < 0 || !ld_ok(n, lda) || !info || (n > 0 && !A)) return GPC_ERR_ARG;
    h->fell_back = 0;
    const bool mixed = h->opt.precision == GPC_MIXED;
    if (!mixed || !h->opt.mixed_fallback || n == 0) return factor_impl(h, n, A, lda, info, mixed);
    hipStream_t s = h->stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    GPC_HIP(h, hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return GPC_ERR_CAPTURE;   // it copies, allocates and waits
    const size_t bytes = sizeof(double) * (size_t)n * (size_t)n;
    if (bytes > h->acopy_bytes) {
        if (h->acopy) {
            GPC_HIP(h, hipStreamSynchronize(s));
            GPC_HIP(h, hipFree(h->acopy));
            h->acopy = nullptr;
            h->acopy_bytes = 0;
        }
        const hipError_t e = hipMalloc((void**)&h->acopy, bytes);
        if (e != hipSuccess) {
            snprintf(h->err, sizeof(h->err), "copy of A, %zu bytes: %s", bytes, hipGetErrorString(e));
            h->acopy = nullptr;
            return GPC_ERR_ALLOC;
        }
        h->acopy_bytes = bytes;
    }
    const size_t row = sizeof(double) * (size_t)n;
    GPC_HIP(h, hipMemcpy2DAsync(h->acopy, row, A, sizeof(double) * lda, row, n, hipMemcpyDeviceToDevice, s));
    gpc_status st = factor_impl(h, n, A, lda, info, true);
    if (st != GPC_OK) return st;
    int32_t info_h = 0;
    GPC_HIP(h, hipMemcpyAsync(&info_h, info, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GPC_HIP(h, hipStreamSynchronize(s));
    if (info_h == 0) return GPC_OK;
    // the FP32 trailing updates lost definiteness: start again in FP64
    GPC_HIP(h, hipMemcpy2DAsync(A, sizeof(double) * lda, h->acopy, row, row, n, hipMemcpyDeviceToDevice, s));
    h->fell_back = 1;
    return factor_impl(h, n, A, lda, info, false);
}

gpc_status gpc_get_fallback(const gpc_handle* h, int32_t* fell_back)
{
    if (!h || !fell_back) return GPC_ERR_ARG;
    *fell_back = h->fell_back;
    return GPC_OK;
}

gpc_status gpc_factor_noalloc(gpc_handle* h, int64_t n, double* A, int64_t lda, int32_t* info)
{
    if (!h || n < 0 || !ld_ok(n, lda) || !info || (n > 0 && !A)) return GPC_ERR_ARG;
    if (h->opt.precision != GPC_FP64) {
        snprintf(h->err, sizeof(h->err), "gpc_factor_noalloc: FP64 only (the mixed form needs n-sized panels)");
        return GPC_ERR_ARG;
    }
    double* linv = scratch_ptr(h, h->device);
    if (!linv) return GPC_ERR_HIP;
    h->fell_back = 0;
    const bool tr = h->trace;
    h->trace = false;   // launch tracing takes events from a pool that may grow
    const gpc_status st = factor_impl(h, n, A, lda, info, false, linv);
    h->trace = tr;
    return st;
}

// --------------------------------------------------------------- adjoint ---
// Blocked reverse sweep (section 3.3.2), diagonal blocks from last to first.
// With D = L[j:k, j:k], R = L[j:k, 0:j], C = L[k:n, j:k], B = L[k:n, 0:j] and
// the matching blocks of Lbar (Dbar, Rbar, Cbar, Bbar):
//   Cbar <- Cbar D^-1;  Bbar -= Cbar R;  Dbar <- tril(Dbar - Cbar^T C);
//   P = D^T Dbar;  S = tril(P) + stril(P)^T;  M = D^-T S D^-1  (symmetric);
//   Rbar -= Cbar^T B + M R;  Dbar <- tril(M) - diag(M)/2.
// The D^-1 of every block come from launches up front; the long products
// Cbar^T C and [M; Cbar]^T [R; B] (inner dimension n-j) are split along k into
// fixed slices that are added in a fixed order.
//
// Schedule of step q (block columns [j, k)): the "chain" (panel solve,
// Cbar^T C, diagonal step) feeds the updates of Bbar and Rbar, which are split
// into the next block's columns [j-b, j) ("narrow", needed by step q-1's
// chain) and the rest [0, j-b) ("big").  With lookahead the big updates run on
// a second stream:
//   main: wait big(q+2); chain(q); record chain(q); wait big(q+1); narrow(q)
//   side: wait chain(q); big(q); record big(q)
// chain(q) reads columns that big(q+1) does not write; narrow(q) writes
// columns big(q+1) writes.  In a group of steps the earlier steps' big(q)
// hold only their Rbar updates and the group's last step's big the Bbar
// updates of all of them; the rules above still order every access (each
// step's chain reads only its own block's columns, and its narrow launch
// applies every term still pending for them).  The FP32 copies of M read by
// big(q) are double-buffered by step parity and those of Cbar by group
// parity (the first chain of the group after next, the next writer of the
// same buffer, waits for a big(q') with q' no larger than the group's last
// step); narrow and big use separate slice buffers.
gpc_status gpc_adjoint(gpc_handle* h, int64_t n, const double* L, int64_t ldl, double* Lbar,
                       int64_t ldlb)
{
    if (!h || n < 0 || !ld_ok(n, ldl) || !ld_ok(n, ldlb) || (n > 0 && (!L || !Lbar)))
        return GPC_ERR_ARG;
    if (overlap(L, n, n, ldl, Lbar, n, n, ldlb)) return GPC_ERR_ARG;
    if (n == 0) return GPC_OK;
    hipStream_t s = h->stream;
    // 512-blocks from n = 8192 in both forms (half the steps: taller row
    // updates, fewer split-K slices and chain launches), else 256; an explicit
    // block option up to 512
    const int b = h->opt.block > 0 ? std::min(h->opt.block, 2 * kDefaultBlock)
                                   : (n >= 8192 ? 2 * kDefaultBlock : kDefaultBlock);
    const int64_t nblk = (n + b - 1) / b;
    const int kMaxSd = 64, kMaxSr = 32;
    const bool mixed = h->opt.precision == GPC_MIXED;
    const bool la = h->opt.lookahead != 0 && nblk > 2;
    auto tiles128 = [](int64_t M, int64_t N) { return ((M + 127) / 128) * ((N + 127) / 128); };
    // Groups of G steps: q0 = nblk-2, nblk-2-G, ... down to q_lo = max(1,
    // q0-G+1).  Step q of a group applies its Bbar update to the next block's
    // columns together with the updates still pending from the group's
    // earlier steps q+1 .. q0 (Cbar columns [j, j + P b) of Lbar against rows
    // [j, j + P b) of L, P = q0 - q + 1); the group's last step applies all of
    // them to the other columns too, so the big products run at K = G b.
    // Row block r of such a product (counted from its first row) takes the
    // terms of steps q .. q+r only: its k stops at (r+1) b, where the operand
    // would run into the diagonal blocks and the strict upper triangle.
    // default: pairs below 512-blocks (the big products then run at K = 512)
    const int G = b % 128 == 0 ? (h->opt.adjoint_group > 0 ? h->opt.adjoint_group : (b >= 512 ? 1 : kDefaultAdjGroup))
                               : 1;
    auto in_group = [&](int64_t q) { return q >= 1 && q <= nblk - 2; };
    auto gtop = [&](int64_t q) { return q + (nblk - 2 - q) % G; };
    auto glow = [&](int64_t q) { return std::max<int64_t>(1, gtop(q) - G + 1); };
    // the FP32 panel copies of one group share a buffer; groups alternate
    // between two (the last step, which has none, and step 0 count as groups)
    std::vector<uint8_t> gpar((size_t)nblk, 0);
    for (int64_t q = 0; q < nblk; ++q) {
        const int64_t gi = in_group(q) ? (nblk - 2 - q) / G : (q == 0 ? (nblk - 2) / G + 1 : -1);
        gpar[(size_t)q] = (uint8_t)(gi & 1);
    }

    // plan the split counts of every step to size the slice buffers
    int64_t prn_elems = 1, prb_elems = 1;
    for (int64_t q = nblk - 1; q >= 1; --q) {
        const int64_t j = q * b, k = std::min<int64_t>(n, j + b), bq = k - j, K = bq + (n - k);
        const int64_t bn = std::min<int64_t>(b, j), jb = j - bn;
        int sr; int64_t ch;
        splitk_plan(tiles128(bq, bn), K, kMaxSr, 2 * (int64_t)h->cus, &sr, &ch);
        prn_elems = std::max<int64_t>(prn_elems, (int64_t)sr * bq * bn);
        if (jb > 0) {
            splitk_plan(tiles128(bq, jb), K, kMaxSr, 2 * (int64_t)h->cus, &sr, &ch);
            prb_elems = std::max<int64_t>(prb_elems, (int64_t)sr * bq * jb);
        }
    }
    const size_t bb = (size_t)b * b;
    const size_t n_dinv = (size_t)nblk * bb;
    const size_t n_pd = std::max((size_t)kMaxSd * bb, (size_t)nblk * (b / 2) * (b / 2));
    const size_t n_dbl = n_dinv + n_pd + 5 * bb + (size_t)prn_elems + (size_t)prb_elems;
    // mixed: FP32 copies of the strict lower triangle of L, of the Cbar
    // panels (two buffers of n x G b: step q of a group whose last step is
    // q_lo in columns and rows from (q - q_lo) b, rows counted from q_lo's
    // first Cbar row) and (two) of M: the FP32 operands of the updates
    const int64_t ldf = n, ldcp = (int64_t)G * b;
    const size_t n_flt = mixed ? (size_t)n * n + 2 * (size_t)n * ldcp + 2 * bb : 0;
    gpc_status st = ensure_ws(h, sizeof(double) * n_dbl + sizeof(float) * n_flt);
    if (st != GPC_OK) return st;
    double* Dinv = (double*)h->ws;
    double* Pd = Dinv + n_dinv;
    double* Wd = Pd + n_pd;
    double* Sw = Wd + bb;
    double* Tw = Sw + bb;
    double* Mw2 = Tw + bb;           // two b x b buffers
    double* Prn = Mw2 + 2 * bb;
    double* Prb = Prn + prn_elems;
    float* Lf = (float*)(Prb + prb_elems);
    float* Cf2 = Lf + (size_t)n * n;
    float* Mf2 = Cf2 + 2 * (size_t)n * ldcp;
    if (mixed) GPC_HIP(h, convert_lower_f32(s, n, L, ldl, Lf, ldf));

    {
        const double db = (double)b;
        Traced t(h, GPC_K_DIAG_INVERSE, (double)nblk * db * db * db / 3.0, 8.0 * 2.0 * (double)nblk * db * db);
        GPC_HIP(h, diag_block_inverses(s, n, b, L, ldl, Dinv, Pd));   // Pd is free until the sweep
    }
    hipStream_t s2 = s;
    if (la) {
        if (!h->side) GPC_HIP(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        s2 = h->side;
        hipEvent_t e0 = sync_event(h, 0);
        if (!e0 || !sync_event(h, 2 + 2 * (size_t)nblk)) return GPC_ERR_HIP;
        GPC_HIP(h, hipEventRecord(e0, s));
        GPC_HIP(h, hipStreamWaitEvent(s2, e0, 0));
        // the sweep reads no element of Lbar's strict upper triangle and
        // writes none but with zeros: clear it on the side stream at the start
        GPC_HIP(h, zero_strict_upper(s2, n, Lbar, ldlb));
    }
    auto ev_chain = [&](int64_t q) { return sync_event(h, 1 + 2 * (size_t)q); };
    auto ev_big = [&](int64_t q) { return sync_event(h, 2 + 2 * (size_t)q); };

    for (int64_t q = nblk - 1; q >= 0; --q) {
        const int64_t j = q * b, k = std::min<int64_t>(n, j + b), bq = k - j, nr = n - k;
        const double* D = L + j * ldl + j;
        const double* Dq_inv = Dinv + (size_t)q * bb;
        double* Dbar = Lbar + j * ldlb + j;
        double* Cbar = Lbar + k * ldlb + j;
        const double* C = L + k * ldl + j;
        double* Mw = Mw2 + (q & 1) * bb;
        const bool grp = in_group(q);
        const int64_t P = grp ? gtop(q) - q + 1 : 1;          // steps whose Bbar terms this step applies
        const bool defer = grp && q > glow(q);                // the group's later step applies the rest
        const int64_t go = grp ? (q - glow(q)) * b : 0;       // this step's place in the group's buffer
        float* Cf = Cf2 + gpar[(size_t)q] * (size_t)n * ldcp + (size_t)go * ldcp + go;
        float* Mf = Mf2 + (q & 1) * bb;
        const double dbq = (double)bq, dnr = (double)nr;
        if (la && q + 2 <= nblk - 1) GPC_HIP(h, hipStreamWaitEvent(s, ev_big(q + 2), 0));
        // ---- chain
        int sd = 0;
        if (nr > 0) {
            {
                Traced t(h, GPC_K_ADJ_PANEL_SOLVE, dnr * dbq * dbq, 8.0 * (2.0 * dnr * dbq + dbq * dbq));
                // Cbar <- Cbar D^-1 in place, 128 output columns per launch from
                // the left: output columns [c0, c0 + w) read the columns from c0
                // on (D^-1 is lower), which no earlier launch has written.
                for (int64_t c0 = 0; c0 < bq; c0 += kDiagMax) {
                    const int64_t w = std::min<int64_t>(kDiagMax, bq - c0);
                    GemmArgs g5 = gemm_args(nr, w, bq - c0, Cbar + c0, ldlb, Dq_inv + c0 * b + c0, b, Cbar + c0, ldlb);
                    if (mixed) {
                        g5.Cf = Cf + c0;
                        g5.ldcf = ldcp;
                    }
                    GPC_HIP(h, gemm_f64(s, panel_tile(nr, h->cus), false, false, EPI_STORE, false, g5, 1));
                }
            }
            int64_t ch;
            splitk_plan(((bq + 63) / 64) * ((bq + 63) / 64), nr, kMaxSd, 4 * (int64_t)h->cus, &sd, &ch);
            Traced t(h, GPC_K_ADJ_DIAG_PRODUCT, 2.0 * dbq * dbq * dnr, 8.0 * (2.0 * dnr * dbq + sd * dbq * dbq));
            GemmArgs gd = gemm_args(bq, bq, nr, Cbar, ldlb, C, ldl, Pd, bq);
            gd.kchunk = ch;
            gd.pstride = (int64_t)bb;
            GPC_HIP(h, gemm_f64(s, TILE_64, true, false, EPI_PARTIAL, false, gd, sd));
        }
        {
            Traced t(h, GPC_K_ADJ_DIAG_BLOCK, 3.0 * dbq * dbq * dbq, 8.0 * 8.0 * dbq * dbq);
            GPC_HIP(h, reduce_tril(s, (int)bq, Dbar, ldlb, Pd, sd, (int64_t)bb, Wd));
            // S = sym(D^T W), T = S D^-1, M = D^-T T: three dependent bq^3
            // products of only (bq/64)^2 output tiles each, so K is split in
            // 64-row slices (partial sums in Pd, free again after reduce_tril)
            // and a reduction applies each product's epilogue.  T is formed
            // as its transpose D^-T S (S is symmetric), so that all three
            // products read their A operand k-major.
            const int sk = (int)std::max<int64_t>(1, (bq + 63) / 64);
            auto part = [&](const double* A, int64_t lda, const double* B, int64_t ldbb, int alow) -> hipError_t {
                GemmArgs g = gemm_args(bq, bq, bq, A, lda, B, ldbb, Pd, bq);
                g.a_lower = alow;
                g.kchunk = 64;
                g.pstride = (int64_t)bb;
                return gemm_f64(s, TILE_64, true, false, EPI_PARTIAL, false, g, sk);
            };
            GPC_HIP(h, part(D, ldl, Wd, bq, 1));
            GPC_HIP(h, reduce_epi(s, (int)bq, Pd, sk, (int64_t)bb, 0, Sw, bq, nullptr, 0, nullptr, 0));
            GPC_HIP(h, part(Dq_inv, b, Sw, bq, 0));
            GPC_HIP(h, reduce_epi(s, (int)bq, Pd, sk, (int64_t)bb, 1, Tw, bq, nullptr, 0, nullptr, 0));
            GPC_HIP(h, part(Dq_inv, b, Tw, bq, 0));
            GPC_HIP(h, reduce_epi(s, (int)bq, Pd, sk, (int64_t)bb, 2, Mw, bq, mixed ? Mf : nullptr, bq, Dbar, ldlb));
        }
        if (j == 0) continue;
        // ---- updates of Bbar and Rbar, columns [c0, c0 + nc)
        const int64_t K = bq + nr;
        // this step's Bbar term and the pending ones of steps q+1 .. q+P-1
        // (Cbar columns [j, j + P b) against L rows [j, j + P b)), row block
        // r of the product taking P' = min(P, r + 1) of them
        auto left = [&](hipStream_t qs, int64_t c0, int64_t nc) -> gpc_status {
            if (nr <= 0 || nc <= 0) return GPC_OK;
            const double dnc = (double)nc, dP = (double)P, kl = dP * dbq;
            // k-products: (P-1) staircase row blocks, then the full ones
            const double kprod = dbq * dbq * dP * (dP - 1.0) / 2.0 + (dnr - (dP - 1.0) * dbq) * dP * dbq;
            Traced t(h, GPC_K_ADJ_LEFT_UPDATE, 2.0 * dnc * kprod,
                     16.0 * dnr * dnc + (mixed ? 4.0 : 8.0) * kl * (dnr + dnc), qs);
            const int64_t K6 = P * bq;
            GemmArgs g6 = mixed ? gemm_args(nr, nc, K6, Cf, ldcp, Lf + j * ldf + c0, ldf, Lbar + k * ldlb + c0, ldlb)
                                : gemm_args(nr, nc, K6, Cbar, ldlb, L + j * ldl + c0, ldl, Lbar + k * ldlb + c0, ldlb);
            if (P > 1) g6.kstep = bq;
            if (mixed) GPC_HIP(h, gemm_f32in(qs, TILE_128, false, false, EPI_SUB, false, g6, 1));
            else GPC_HIP(h, gemm_f64(qs, TILE_128, false, false, EPI_SUB, false, g6, 1));
            return GPC_OK;
        };
        auto rowupd = [&](hipStream_t qs, int64_t c0, int64_t nc, double* Pbuf) -> gpc_status {
            if (nc <= 0) return GPC_OK;
            const double dnc = (double)nc;
            int sr; int64_t ch;
            splitk_plan(tiles128(bq, nc), K, kMaxSr, 2 * (int64_t)h->cus, &sr, &ch);
            {
                Traced t(h, GPC_K_ADJ_ROW_UPDATE, 2.0 * dbq * dnc * (double)K,
                         (mixed ? 4.0 : 8.0) * (double)K * (dbq + dnc) + 8.0 * sr * dbq * dnc, qs);
                if (mixed) {
                    GemmArgs gr = gemm_args(bq, nc, K, Cf, ldcp, Lf + j * ldf + c0, ldf, Pbuf, nc);
                    gr.Ahead = Mf;
                    gr.ldah = bq;
                    gr.head_k = bq;
                    gr.kchunk = ch;
                    gr.pstride = bq * nc;
                    GPC_HIP(h, gemm_f32in(qs, TILE_128, true, false, EPI_PARTIAL, false, gr, sr));
                } else {
                    GemmArgs gr = gemm_args(bq, nc, K, Cbar, ldlb, L + j * ldl + c0, ldl, Pbuf, nc);
                    gr.Ahead = Mw;
                    gr.ldah = bq;
                    gr.head_k = bq;
                    gr.kchunk = ch;
                    gr.pstride = bq * nc;
                    GPC_HIP(h, gemm_f64(qs, TILE_128, true, false, EPI_PARTIAL, false, gr, sr));
                }
            }
            Traced t(h, GPC_K_REDUCE, dbq * dnc * sr, 8.0 * (sr + 2.0) * dbq * dnc, qs);
            GPC_HIP(h, reduce_sub(qs, bq, nc, Pbuf, sr, bq * nc, Lbar + j * ldlb + c0, ldlb));
            return GPC_OK;
        };
        const int64_t bn = std::min<int64_t>(b, j), jb = j - bn;
        if (la) {
            GPC_HIP(h, hipEventRecord(ev_chain(q), s));
            GPC_HIP(h, hipStreamWaitEvent(s2, ev_chain(q), 0));
            if (!defer && (st = left(s2, 0, jb)) != GPC_OK) return st;
            if ((st = rowupd(s2, 0, jb, Prb)) != GPC_OK) return st;
            GPC_HIP(h, hipEventRecord(ev_big(q), s2));
            if (q + 1 <= nblk - 1) GPC_HIP(h, hipStreamWaitEvent(s, ev_big(q + 1), 0));
        }
        if ((st = left(s, jb, bn)) != GPC_OK) return st;
        if ((st = rowupd(s, jb, bn, Prn)) != GPC_OK) return st;
        if (!la) {
            if (!defer && (st = left(s, 0, jb)) != GPC_OK) return st;
            if ((st = rowupd(s, 0, jb, Prb)) != GPC_OK) return st;
        }
    }
    if (la) {   // join the side stream
        hipEvent_t ej = sync_event(h, 0);
        GPC_HIP(h, hipEventRecord(ej, s2));
        GPC_HIP(h, hipStreamWaitEvent(s, ej, 0));
    } else {
        GPC_HIP(h, zero_strict_upper(s, n, Lbar, ldlb));
    }
    return GPC_OK;
}

// ----------------------------------------------------------------- solves ---
gpc_status gpc_trsm(gpc_handle* h, int32_t trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                    double* B, int64_t ldb)
{
    if (!h || (trans != GPC_NOTRANS && trans != GPC_TRANS) || n < 0 || nrhs < 0 || !ld_ok(n, ldl) ||
        !ld_ok(nrhs, ldb) || (n > 0 && nrhs > 0 && (!L || !B)))
        return GPC_ERR_ARG;
    if (overlap(L, n, n, ldl, B, n, nrhs, ldb)) return GPC_ERR_ARG;
    if (n == 0 || nrhs == 0) return GPC_OK;
    hipStream_t s = h->stream;
    const int b = solve_block(n);
    const int64_t nblk = (n + b - 1) / b;
    const size_t n_dinv = (size_t)nblk * b * b;
    gpc_status st = ensure_ws(h, sizeof(double) * (2 * n_dinv + (size_t)trsm_workspace(n)));
    if (st != GPC_OK) return st;
    double* Dinv = (double*)h->ws;
    double* Cpl = Dinv + n_dinv;
    double* Y = Cpl + n_dinv;
    GPC_HIP(h, diag_block_inverses(s, n, b, L, ldl, Dinv, Cpl));
    GPC_HIP(h, trsm_couplings(s, trans, n, L, ldl, Dinv, b, Cpl));
    GPC_HIP(h, trsm_blocked(s, trans, n, nrhs, L, ldl, Dinv, Cpl, b, B, ldb, Y, h->cus, h->opt.test_flags, h->status_dev));
    return GPC_OK;
}

gpc_status gpc_logdet(gpc_handle* h, int64_t n, const double* L, int64_t ldl, double* out)
{
    if (!h || n < 0 || !ld_ok(n, ldl) || !out || (n > 0 && !L)) return GPC_ERR_ARG;
    GPC_HIP(h, logdet(h->stream, n, L, ldl, out));
    return GPC_OK;
}

// --------------------------------------------------------------- GP -------
gpc_status gpc_gp_kgen_se(gpc_handle* h, int64_t n, int32_t d, const double* X, const double* theta,
                          double* K, int64_t ldk)
{
    if (!h || n < 0 || d < 1 || d > kMaxGpDim || !ld_ok(n, ldk) || (n > 0 && (!X || !theta || !K)))
        return GPC_ERR_ARG;
    GPC_HIP(h, gp_kgen_se(h->stream, n, d, X, theta, K, ldk));
    return GPC_OK;
}

gpc_status gpc_gp_value(gpc_handle* h, int64_t n, const double* L, int64_t ldl, const double* y, double* z,
                        double* alpha, double* logdet_out, double* f_out)
{
    if (!h || n < 0 || !ld_ok(n, ldl) || !logdet_out || !f_out || (n > 0 && (!L || !y || !z || !alpha)))
        return GPC_ERR_ARG;
    if (overlap(z, 1, n, n, alpha, 1, n, n) || overlap(z, 1, n, n, L, n, n, ldl) ||
        overlap(alpha, 1, n, n, L, n, n, ldl) || overlap(z, 1, n, n, y, 1, n, n) ||
        overlap(alpha, 1, n, n, y, 1, n, n))
        return GPC_ERR_ARG;
    hipStream_t s = h->stream;
    if (n > 0) {
        const int b = solve_block(n);
        const int64_t nblk = (n + b - 1) / b;
        const size_t n_dinv = (size_t)nblk * b * b;
        gpc_status st = ensure_ws(h, sizeof(double) * (3 * n_dinv + (size_t)trsm_workspace(n)));
        if (st != GPC_OK) return st;
        double* Dinv = (double*)h->ws;
        double* Cf = Dinv + n_dinv;
        double* Cb = Cf + n_dinv;
        double* Y = Cb + n_dinv;
        GPC_HIP(h, diag_block_inverses(s, n, b, L, ldl, Dinv, Cf));
        GPC_HIP(h, trsm_couplings(s, 0, n, L, ldl, Dinv, b, Cf));
        GPC_HIP(h, trsm_couplings(s, 1, n, L, ldl, Dinv, b, Cb));
        GPC_HIP(h, vec_copy(s, n, y, z));
        GPC_HIP(h, trsm_blocked(s, 0, n, 1, L, ldl, Dinv, Cf, b, z, 1, Y, h->cus, h->opt.test_flags, h->status_dev));
        GPC_HIP(h, vec_copy(s, n, z, alpha));
        GPC_HIP(h, trsm_blocked(s, 1, n, 1, L, ldl, Dinv, Cb, b, alpha, 1, Y, h->cus, h->opt.test_flags, h->status_dev));
    }
    GPC_HIP(h, logdet(s, n, L, ldl, logdet_out));
    GPC_HIP(h, gp_value(s, n, z, logdet_out, f_out));
    return GPC_OK;
}

gpc_status gpc_gp_value_refined(gpc_handle* h, int64_t n, const double* K, int64_t ldk, const double* L,
                                int64_t ldl, const double* y, double* z, double* alpha, double* logdet_out,
                                double* f_out, int32_t* iters, double* eta)
{
    if (!h || n < 0 || !ld_ok(n, ldk) || !ld_ok(n, ldl) || !logdet_out || !f_out || !iters || !eta ||
        (n > 0 && (!K || !L || !y || !z || !alpha)))
        return GPC_ERR_ARG;
    if (overlap(z, 1, n, n, alpha, 1, n, n) || overlap(z, 1, n, n, L, n, n, ldl) ||
        overlap(z, 1, n, n, K, n, n, ldk) || overlap(z, 1, n, n, y, 1, n, n))
        return GPC_ERR_ARG;
    gpc_status st = gpc_solve_refined(h, n, K, ldk, L, ldl, y, alpha, iters, eta);
    if (st != GPC_OK && st != GPC_ERR_REFINE) return st;
    hipStream_t s = h->stream;
    if (n > 0) {
        // z = L^T alpha from the lower triangle of L: one column of output
        // tiles with the inner dimension split (fixed-order sum)
        int sp = 1;
        int64_t ch = n;
        splitk_plan((n + 127) / 128, n, 32, 2 * (int64_t)h->cus, &sp, &ch);
        if (sp > 1) {
            gpc_status wst = ensure_ws(h, sizeof(double) * (size_t)sp * (size_t)n);
            if (wst != GPC_OK) return wst;
        }
        GemmArgs g = gemm_args(n, 1, n, L, ldl, alpha, 1, sp > 1 ? (double*)h->ws : z, 1);
        g.a_lower = 1;   // read k-major (L^T); the strict upper part of L is never read
        if (sp > 1) {
            g.kchunk = ch;
            g.pstride = n;
            GPC_HIP(h, gemm_f64(s, TILE_128, true, false, EPI_PARTIAL, false, g, sp));
            GPC_HIP(h, reduce_store(s, n, 1, (double*)h->ws, sp, n, 0.0, z, 1));
        } else {
            GPC_HIP(h, gemm_f64(s, TILE_128, true, false, EPI_STORE, false, g, 1));
        }
    }
    GPC_HIP(h, logdet(s, n, L, ldl, logdet_out));
    GPC_HIP(h, gp_value_dot(s, n, y, alpha, logdet_out, f_out));
    return st;
}

gpc_status gpc_gp_lbar(gpc_handle* h, int64_t n, const double* L, int64_t ldl, const double* alpha,
                       const double* z, double* Lbar, int64_t ldlb)
{
    if (!h || n < 0 || !ld_ok(n, ldl) || !ld_ok(n, ldlb) || (n > 0 && (!L || !alpha || !z || !Lbar)))
        return GPC_ERR_ARG;
    if (overlap(Lbar, n, n, ldlb, L, n, n, ldl) || overlap(Lbar, n, n, ldlb, alpha, 1, n, n) ||
        overlap(Lbar, n, n, ldlb, z, 1, n, n))
        return GPC_ERR_ARG;
    GPC_HIP(h, gp_lbar(h->stream, n, L, ldl, alpha, z, Lbar, ldlb));
    return GPC_OK;
}

gpc_status gpc_gp_hypergrad_se(gpc_handle* h, int64_t n, int32_t d, const double* X, const double* theta,
                               const double* Abar, int64_t ldab, const double* scale, double* grad)
{
    if (!h || n < 0 || d < 1 || d > kMaxGpDim || !ld_ok(n, ldab) || !theta || !grad ||
        (n > 0 && (!X || !Abar)))
        return GPC_ERR_ARG;
    gpc_status st = ensure_ws(h, sizeof(double) * (size_t)gp_hypergrad_parts(n, d));
    if (st != GPC_OK) return st;
    GPC_HIP(h, gp_hypergrad_se(h->stream, n, d, X, theta, Abar, ldab, scale, grad, (double*)h->ws));
    return GPC_OK;
}

// ------------------------------------------------------------ refinement ---
// Solve K x = y with a factor L of (an approximation of) K: x_0 = 0, then
// repeat  d = L^-T L^-1 r,  x += d,  r = y - K x  (FP64, K from its lower
// triangle),  eta = |r|_inf / (|K|_inf |x|_inf + |y|_inf)  until eta <= tol.
gpc_status gpc_solve_refined(gpc_handle* h, int64_t n, const double* K, int64_t ldk, const double* L,
                             int64_t ldl, const double* y, double* x, int32_t* iters, double* eta)
{
    if (!h || n < 0 || !ld_ok(n, ldk) || !ld_ok(n, ldl) || !iters || !eta ||
        (n > 0 && (!K || !L || !y || !x)))
        return GPC_ERR_ARG;
    if (overlap(x, 1, n, n, K, n, n, ldk) || overlap(x, 1, n, n, L, n, n, ldl) || overlap(x, 1, n, n, y, 1, n, n))
        return GPC_ERR_ARG;
    hipStream_t s = h->stream;
    if (n == 0) {
        GPC_HIP(h, fill_i32(s, iters, 0));
        GPC_HIP(h, vec_zero(s, 1, eta));
        return GPC_OK;
    }
    const int b = solve_block(n);
    const int64_t nblk = (n + b - 1) / b;
    const size_t n_dinv = (size_t)nblk * b * b;
    const size_t n_part = (size_t)symv_parts(n);
    gpc_status st =
        ensure_ws(h, sizeof(double) * (3 * n_dinv + (size_t)trsm_workspace(n) + 2 * n_part + 3 * (size_t)n));
    if (st != GPC_OK) return st;
    double* Dinv = (double*)h->ws;
    double* Cf = Dinv + n_dinv;
    double* Cb = Cf + n_dinv;
    double* Y = Cb + n_dinv;
    double* part = Y + trsm_workspace(n);
    double* rowabs = part + 2 * n_part;
    double* r = rowabs + n;
    double* d = r + n;
    GPC_HIP(h, diag_block_inverses(s, n, b, L, ldl, Dinv, Cf));
    GPC_HIP(h, trsm_couplings(s, 0, n, L, ldl, Dinv, b, Cf));
    GPC_HIP(h, trsm_couplings(s, 1, n, L, ldl, Dinv, b, Cb));
    GPC_HIP(h, vec_zero(s, n, x));
    GPC_HIP(h, vec_copy(s, n, y, r));
    const int maxit = std::max(1, h->opt.refine_maxit);
    double eta_h = 1.0;
    int it = 0;
    while (it < maxit) {
        ++it;
        GPC_HIP(h, vec_copy(s, n, r, d));
        GPC_HIP(h, trsm_blocked(s, 0, n, 1, L, ldl, Dinv, Cf, b, d, 1, Y, h->cus, h->opt.test_flags, h->status_dev));
        GPC_HIP(h, trsm_blocked(s, 1, n, 1, L, ldl, Dinv, Cb, b, d, 1, Y, h->cus, h->opt.test_flags, h->status_dev));
        GPC_HIP(h, vec_axpy(s, n, d, x));
        if (it == 1)   // the row sums of |K| for eta come from the same pass over K
            GPC_HIP(h, symv_lower_abs(s, n, K, ldk, x, y, -1.0, r, rowabs, part));
        else
            GPC_HIP(h, symv_lower(s, n, K, ldk, x, 0, y, -1.0, r, part));
        GPC_HIP(h, refine_eta(s, n, r, x, y, rowabs, eta));
        uint32_t rec = 0;
        GPC_HIP(h, hipMemcpyAsync(&eta_h, eta, sizeof(double), hipMemcpyDeviceToHost, s));
        GPC_HIP(h, hipMemcpyAsync(&rec, h->status_dev, sizeof(rec), hipMemcpyDeviceToHost, s));
        GPC_HIP(h, hipStreamSynchronize(s));
        if (rec != 0) {   // a sweep ran out of time: x is not a solution
            GPC_HIP(h, fill_i32(s, (int32_t*)h->status_dev, 0));
            GPC_HIP(h, fill_i32(s, iters, it));
            return GPC_ERR_SWEEP;
        }
        if (eta_h <= h->opt.refine_tol) break;
    }
    GPC_HIP(h, fill_i32(s, iters, it));
    return eta_h <= h->opt.refine_tol ? GPC_OK : GPC_ERR_REFINE;
}

// --------------------------------------------------------------- batched ---
namespace {

gpc_status run_batched(gpc_handle* h, int mode, int32_t nb, const int32_t* n_host, const int64_t* off_host,
                       double* A, double* Lb, int32_t* info)
{
    if (!h || nb < 0 || (nb > 0 && (!n_host || !off_host || !A))) return GPC_ERR_ARG;
    if ((mode & 1) && nb > 0 && !info) return GPC_ERR_ARG;
    if ((mode & 2) && nb > 0 && !Lb) return GPC_ERR_ARG;
    for (int32_t i = 0; i < nb; ++i)
        if (n_host[i] < 0 || off_host[i] < 0) return GPC_ERR_ARG;
    if (nb == 0) return GPC_OK;
    if (h->opt.precision == GPC_MIXED) mode |= 4;   // FP32 trailing and B-bar / R-bar products
    hipStream_t s = h->stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    GPC_HIP(h, hipStreamIsCapturing(s, &cs));
    const bool capturing = cs != hipStreamCaptureStatusNone;
    std::vector<int32_t> blocks(h->tune_block, h->tune_block + kTuneBuckets);
    int schedule = h->opt.batched_schedule;
    if (schedule == 0) schedule = *std::max_element(n_host, n_host + nb) >= kGroupedMinN ? 2 : 1;
    BatchPlan* p = h->plan;
    const bool same = p && p->mode == mode && p->A == A && p->Lb == Lb && p->info == info &&
                      p->blocks == blocks && p->schedule == schedule && p->n.size() == (size_t)nb &&
                      std::equal(p->n.begin(), p->n.end(), n_host) && std::equal(p->off.begin(), p->off.end(), off_host);
    if (!same) {
        // a new plan waits for the stream and allocates: not possible while
        // the caller captures
        if (capturing) {
            snprintf(h->err, sizeof(h->err),
                     "no batched plan for these sizes, offsets and pointers: make the same call once before capturing");
            return GPC_ERR_CAPTURE;
        }
        GPC_HIP(h, hipStreamSynchronize(s));
        retire_plan(h);
        h->plan = p = new BatchPlan();
        p->mode = mode;
        p->A = A;
        p->Lb = Lb;
        p->info = info;
        p->n.assign(n_host, n_host + nb);
        p->off.assign(off_host, off_host + nb);
        p->blocks = blocks;
        p->schedule = schedule;
        std::vector<gpc::BatchTask> tasks(nb);
        for (int32_t i = 0; i < nb; ++i) {
            tasks[i].n = n_host[i];
            tasks[i].block = h->tune_block[bucket_of(n_host[i])];
            tasks[i].idx = i;
            tasks[i].pad = 0;
            tasks[i].off = off_host[i];
            const double dn = (double)n_host[i];
            p->flops += ((mode & 1) ? dn * dn * dn / 3.0 + dn * dn / 2.0 + dn / 6.0 : 0.0) +
                        ((mode & 2) ? 2.0 * dn * dn * dn / 3.0 : 0.0);
        }
        std::stable_sort(tasks.begin(), tasks.end(),
                         [](const gpc::BatchTask& a, const gpc::BatchTask& b) { return a.n > b.n; });
        if (schedule == 2) {
            hipError_t ge = hipSuccess;
            p->grouped = gpc::grouped_prepare(nb, tasks.data(), A, Lb, info, mode, &ge);
            if (!p->grouped) return hip_fail(h, ge, "grouped batched schedule");
        } else {
            p->wgs = std::min<int>(nb, 2 * h->cus);
            GPC_HIP(h, hipMalloc(&p->d_tasks, sizeof(gpc::BatchTask) * nb));
            GPC_HIP(h, hipMalloc(&p->d_counter, sizeof(int32_t)));
            GPC_HIP(h, hipMalloc(&p->d_ws, sizeof(double) * gpc::batched_scratch_doubles(p->wgs)));
            GPC_HIP(h, hipMemcpy(p->d_tasks, tasks.data(), sizeof(gpc::BatchTask) * nb, hipMemcpyHostToDevice));
        }
        if (!h->cap_stream) GPC_HIP(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        if (schedule == 2 && !h->side) GPC_HIP(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        GPC_HIP(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        // the grouped schedule's zero fills become a parallel branch of the graph
        hipError_t le = schedule == 2 ? gpc::grouped_enqueue(p->grouped, h->cap_stream, h->side, info)
                                      : gpc::batched_launch(h->cap_stream, nb, p->d_tasks, A, Lb, info, p->d_counter,
                                                            p->d_ws, p->wgs, mode);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(h->cap_stream, &g);
        p->graph = g;
        if (le != hipSuccess) return hip_fail(h, le, "batched launch (capture)");
        if (ce != hipSuccess) return hip_fail(h, ce, "hipStreamEndCapture");
        GPC_HIP(h, hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    }
    Traced t(h, GPC_K_BATCHED, p->flops, 0.0);
    if (!capturing) {
        GPC_HIP(h, hipGraphLaunch(p->exec, s));
    } else {
        // the caller is capturing: record the launch into its graph instead;
        // the plan's buffers then stay allocated until gpc_destroy
        p->pinned = true;
        if (p->schedule == 2) GPC_HIP(h, gpc::grouped_enqueue(p->grouped, s, nullptr, info));
        else GPC_HIP(h, gpc::batched_launch(s, nb, p->d_tasks, A, Lb, info, p->d_counter, p->d_ws, p->wgs, mode));
    }
    return GPC_OK;
}

}  // namespace

gpc_status gpc_factor_batched(gpc_handle* h, int32_t nb, const int32_t* n_host, const int64_t* off_host,
                              double* base, int32_t* info_dev)
{
    return run_batched(h, 1, nb, n_host, off_host, base, nullptr, info_dev);
}

gpc_status gpc_adjoint_batched(gpc_handle* h, int32_t nb, const int32_t* n_host, const int64_t* off_host,
                               const double* Lbase, double* Lbarbase)
{
    return run_batched(h, 2, nb, n_host, off_host, const_cast<double*>(Lbase), Lbarbase, nullptr);
}

gpc_status gpc_factor_adjoint_batched(gpc_handle* h, int32_t nb, const int32_t* n_host, const int64_t* off_host,
                                      double* base, double* Lbarbase, int32_t* info_dev)
{
    return run_batched(h, 3, nb, n_host, off_host, base, Lbarbase, info_dev);
}

// Autotuner of the batched path: for each size bucket, time factor+adjoint of
// a synthetic batch (16 matrices at the bucket's middle order) with inner
// blocks 32 and 64 (median of 3 runs each), keep the faster; optionally
// append the choices to a cache file read by later handles.
gpc_status gpc_autotune_batched(gpc_handle* h, const char* cache_path)
{
    if (!h) return GPC_ERR_ARG;
    hipStream_t s = h->stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    GPC_HIP(h, hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return GPC_ERR_CAPTURE;
    const int mids[kTuneBuckets] = {80, 192, 384, 768, 1024};
    const int cnt = 16;
    // the inner block belongs to the persistent schedule: time that one
    struct ScheduleGuard {
        gpc_handle* h;
        int32_t saved;
        ~ScheduleGuard() { h->opt.batched_schedule = saved; }
    } guard{h, h->opt.batched_schedule};
    h->opt.batched_schedule = 1;
    for (int bk = 0; bk < kTuneBuckets; ++bk) {
        const int64_t n = mids[bk];
        std::vector<int32_t> ns(cnt, (int32_t)n);
        std::vector<int64_t> offs(cnt);
        for (int i = 0; i < cnt; ++i) offs[i] = (int64_t)i * n * n;
        double *A = nullptr, *Lb = nullptr;
        int32_t* info = nullptr;
        hipEvent_t e0, e1;
        GPC_HIP(h, hipMalloc(&A, sizeof(double) * cnt * n * n));
        GPC_HIP(h, hipMalloc(&Lb, sizeof(double) * cnt * n * n));
        GPC_HIP(h, hipMalloc(&info, sizeof(int32_t) * cnt));
        GPC_HIP(h, hipEventCreate(&e0));
        GPC_HIP(h, hipEventCreate(&e1));
        float best_ms = 1e30f;
        int best = h->tune_block[bk];
        for (int cand : {32, 64}) {
            h->tune_block[bk] = cand;   // the synthetic batch lies in bucket bk only
            float t[3];
            for (int r = 0; r < 3; ++r) {
                for (int i = 0; i < cnt; ++i) GPC_HIP(h, gpc::spd_test_fill(s, n, A, Lb, offs[i]));
                GPC_HIP(h, hipEventRecord(e0, s));
                gpc_status st = run_batched(h, 3, cnt, ns.data(), offs.data(), A, Lb, info);
                if (st != GPC_OK) return st;
                GPC_HIP(h, hipEventRecord(e1, s));
                GPC_HIP(h, hipEventSynchronize(e1));
                GPC_HIP(h, hipEventElapsedTime(&t[r], e0, e1));
            }
            std::sort(t, t + 3);
            if (t[1] < best_ms) {
                best_ms = t[1];
                best = cand;
            }
        }
        h->tune_block[bk] = best;
        GPC_HIP(h, hipStreamSynchronize(s));
        retire_plan(h);
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        hipFree(A);
        hipFree(Lb);
        hipFree(info);
    }
    h->tuned = true;
    if (cache_path && *cache_path) {
        FILE* f = fopen(cache_path, "w");
        if (f) {
            for (int bk = 0; bk < kTuneBuckets; ++bk)
                fprintf(f, "gfx950 %d %d %d\n", (int)GPC_FP64, kTuneLimits[bk], h->tune_block[bk]);
            fclose(f);
        }
    }
    return GPC_OK;
}

gpc_status gpc_get_tuning(const gpc_handle* h, int32_t* blocks_out, int32_t* tuned)
{
    if (!h || !blocks_out || !tuned) return GPC_ERR_ARG;
    for (int b = 0; b < kTuneBuckets; ++b) blocks_out[b] = h->tune_block[b];
    *tuned = h->tuned ? 1 : 0;
    return GPC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Operations beside the Cholesky path (include/gpchol_ops.h): the triangular
// inverse and the reverse modes of the solve and the inverse (section 3.2),
// products and their reverse mode (section 3.1), the Bernoulli-logit GLM
// (section 3.4).
#include "gpchol_ops.h"

namespace {

bool trans_ok(int32_t t) { return t == 0 || t == 1; }

}  // namespace

extern "C" {

gpc_status gpc_trtri(gpc_handle* h, int64_t n, const double* L, int64_t ldl, double* X, int64_t ldx)
{
    if (!h || n < 0 || !ld_ok(n, ldl) || !ld_ok(n, ldx) || (n > 0 && (!L || !X))) return GPC_ERR_ARG;
    if (overlap(L, n, n, ldl, X, n, n, ldx)) return GPC_ERR_ARG;
    if (n == 0) return GPC_OK;
    const double dn = (double)n;
    Traced tr(h, GPC_K_OPS, dn * dn * dn / 3.0, 16.0 * dn * dn);
    GPC_HIP(h, trtri_full(h->stream, n, L, ldl, X, ldx));
    return GPC_OK;
}

gpc_status gpc_trtri_adjoint(gpc_handle* h, int64_t n, const double* X, int64_t ldx, const double* Xbar,
                             int64_t ldxb, double* Lbar, int64_t ldlb)
{
    if (!h || n < 0 || !ld_ok(n, ldx) || !ld_ok(n, ldxb) || !ld_ok(n, ldlb) || (n > 0 && (!X || !Xbar || !Lbar)))
        return GPC_ERR_ARG;
    if (overlap(Lbar, n, n, ldlb, X, n, n, ldx) || overlap(Lbar, n, n, ldlb, Xbar, n, n, ldxb)) return GPC_ERR_ARG;
    if (n == 0) return GPC_OK;
    gpc_status st = ensure_ws(h, sizeof(double) * (size_t)n * (size_t)n);
    if (st != GPC_OK) return st;
    double* Pt = (double*)h->ws;   // P^T = tril(Xbar)^T X, n x n
    hipStream_t s = h->stream;
    const double dn = (double)n;
    Traced tr(h, GPC_K_OPS, 2.0 * dn * dn * dn, 8.0 * 5.0 * dn * dn);
    GemmArgs g1{};
    g1.M = n; g1.N = n; g1.K = n;
    g1.A = Xbar; g1.lda = ldxb; g1.a_lower = 1;   // read k-major: Xbar^T, its strict upper part masked
    g1.B = X; g1.ldb = ldx;
    g1.C = Pt; g1.ldc = n;
    g1.kchunk = n;
    GPC_HIP(h, gemm_f64(s, TILE_128, true, false, EPI_STORE, false, g1, 1));
    GemmArgs g2{};                                  // Lbar = -tril(P X^T), lower tiles
    g2.M = n; g2.N = n; g2.K = n;
    g2.A = Pt; g2.lda = n;                          // read k-major: (P^T)^T = P
    g2.B = X; g2.ldb = ldx;                         // read n-major: X^T
    g2.C = Lbar; g2.ldc = ldlb;
    g2.kchunk = n;
    g2.negate = 1;
    GPC_HIP(h, gemm_f64(s, TILE_128, true, true, EPI_STORE, true, g2, 1));
    GPC_HIP(h, zero_strict_upper(s, n, Lbar, ldlb));
    return GPC_OK;
}

gpc_status gpc_trsm_adjoint(gpc_handle* h, int32_t trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                            const double* C, int64_t ldc, double* Cbar, int64_t ldcb, double* Lbar, int64_t ldlb)
{
    if (!h || !trans_ok(trans) || n < 0 || nrhs < 0 || !ld_ok(n, ldl) || !ld_ok(nrhs, ldc) || !ld_ok(nrhs, ldcb) ||
        !ld_ok(n, ldlb) || (n > 0 && (!L || !Lbar)) || (n > 0 && nrhs > 0 && (!C || !Cbar)))
        return GPC_ERR_ARG;
    if (overlap(Cbar, n, nrhs, ldcb, L, n, n, ldl) || overlap(Cbar, n, nrhs, ldcb, C, n, nrhs, ldc) ||
        overlap(Lbar, n, n, ldlb, L, n, n, ldl) || overlap(Lbar, n, n, ldlb, C, n, nrhs, ldc) ||
        overlap(Lbar, n, n, ldlb, Cbar, n, nrhs, ldcb))
        return GPC_ERR_ARG;
    if (n == 0) return GPC_OK;
    hipStream_t s = h->stream;
    // Bbar = L^-T Cbar (trans 0) or L^-1 Cbar (trans 1), in place
    gpc_status st = gpc_trsm(h, trans ? GPC_NOTRANS : GPC_TRANS, n, nrhs, L, ldl, Cbar, ldcb);
    if (st != GPC_OK) return st;
    const double dn = (double)n, dr = (double)nrhs;
    Traced tr(h, GPC_K_OPS, dn * (dn + 1.0) * dr, 8.0 * (2.0 * dn * dr + dn * (dn + 1.0) / 2.0));
    // Lbar = -tril(Bbar C^T) (trans 0) or -tril(C Bbar^T) (trans 1): lower tiles
    GemmArgs g{};
    g.M = n; g.N = n; g.K = nrhs;
    g.A = trans ? C : Cbar; g.lda = trans ? ldc : ldcb;
    g.B = trans ? Cbar : C; g.ldb = trans ? ldcb : ldc;
    g.C = Lbar; g.ldc = ldlb;
    g.kchunk = std::max<int64_t>(1, nrhs);
    g.negate = nrhs > 0;                            // no right-hand side: Lbar = +0
    GPC_HIP(h, gemm_f64(s, TILE_128, false, true, EPI_STORE, true, g, 1));
    GPC_HIP(h, zero_strict_upper(s, n, Lbar, ldlb));
    return GPC_OK;
}

gpc_status gpc_gemm(gpc_handle* h, int32_t ta, int32_t tb, int64_t M, int64_t N, int64_t K, const double* A,
                    int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc)
{
    if (!h || !trans_ok(ta) || !trans_ok(tb) || M < 0 || N < 0 || K < 0 || !(beta == 0.0 || beta == 1.0))
        return GPC_ERR_ARG;
    if (!ld_ok(ta ? M : K, lda) || !ld_ok(tb ? K : N, ldb) || !ld_ok(N, ldc)) return GPC_ERR_ARG;
    if (M > 0 && N > 0 && (!C || (K > 0 && (!A || !B)))) return GPC_ERR_ARG;
    if (overlap(C, M, N, ldc, A, ta ? K : M, ta ? M : K, lda) || overlap(C, M, N, ldc, B, tb ? N : K, tb ? K : N, ldb))
        return GPC_ERR_ARG;
    if (M == 0 || N == 0) return GPC_OK;
    const int msp = h->opt.gemm_max_splits > 0 ? h->opt.gemm_max_splits : kGemmMaxSplits;
    const int64_t wsd = gemm_general_workspace(M, N, K, h->cus, msp);
    gpc_status st = ensure_ws(h, sizeof(double) * (size_t)std::max<int64_t>(wsd, 1));
    if (st != GPC_OK) return st;
    const double dM = (double)M, dN = (double)N, dK = (double)K;
    Traced tr(h, GPC_K_OPS, 2.0 * dM * dN * dK, 8.0 * (dM * dK + dK * dN + (beta == 0.0 ? 1.0 : 2.0) * dM * dN));
    int sp = 1;
    GPC_HIP(h, gemm_general(h->stream, ta != 0, tb != 0, M, N, K, A, lda, B, ldb, beta, C, ldc, (double*)h->ws,
                            h->cus, msp, &sp));
    h->last_splits = sp;
    return GPC_OK;
}

gpc_status gpc_gemm_adjoint(gpc_handle* h, int32_t ta, int32_t tb, int64_t M, int64_t N, int64_t K, const double* A,
                            int64_t lda, const double* B, int64_t ldb, const double* Cbar, int64_t ldcb, double beta,
                            double* Abar, int64_t ldab, double* Bbar, int64_t ldbb)
{
    if (!h || !trans_ok(ta) || !trans_ok(tb) || M < 0 || N < 0 || K < 0 || !(beta == 0.0 || beta == 1.0))
        return GPC_ERR_ARG;
    const int64_t ar = ta ? K : M, ac = ta ? M : K;   // stored shape of A
    const int64_t br = tb ? N : K, bc = tb ? K : N;   // stored shape of B
    if (!ld_ok(ac, lda) || !ld_ok(bc, ldb) || !ld_ok(N, ldcb)) return GPC_ERR_ARG;
    if (Abar && !ld_ok(ac, ldab)) return GPC_ERR_ARG;
    if (Bbar && !ld_ok(bc, ldbb)) return GPC_ERR_ARG;
    if (overlap(Abar, ar, ac, ldab, Bbar, br, bc, ldbb) || overlap(Abar, ar, ac, ldab, Cbar, M, N, ldcb) ||
        overlap(Bbar, br, bc, ldbb, Cbar, M, N, ldcb) || overlap(Abar, ar, ac, ldab, B, br, bc, ldb) ||
        overlap(Bbar, br, bc, ldbb, A, ar, ac, lda))
        return GPC_ERR_ARG;
    // op(A) = A:   Abar  = Cbar op(B)^T           op(A) = A^T: Abar = op(B) Cbar^T
    // op(B) = B:   Bbar  = op(A)^T Cbar           op(B) = B^T: Bbar = Cbar^T op(A)
    if (Abar) {
        gpc_status st = ta ? gpc_gemm(h, tb, 1, K, M, N, B, ldb, Cbar, ldcb, beta, Abar, ldab)
                           : gpc_gemm(h, 0, tb ? 0 : 1, M, K, N, Cbar, ldcb, B, ldb, beta, Abar, ldab);
        if (st != GPC_OK) return st;
    }
    if (Bbar) {
        gpc_status st = tb ? gpc_gemm(h, 1, ta, N, K, M, Cbar, ldcb, A, lda, beta, Bbar, ldbb)
                           : gpc_gemm(h, ta ? 0 : 1, 0, K, N, M, A, lda, Cbar, ldcb, beta, Bbar, ldbb);
        if (st != GPC_OK) return st;
    }
    return GPC_OK;
}

gpc_status gpc_multiply_transpose(gpc_handle* h, int64_t M, int64_t K, const double* A, int64_t lda, double* C,
                                  int64_t ldc)
{
    if (!h || M < 0 || K < 0 || !ld_ok(K, lda) || !ld_ok(M, ldc) || (M > 0 && (!C || (K > 0 && !A))))
        return GPC_ERR_ARG;
    if (overlap(C, M, M, ldc, A, M, K, lda)) return GPC_ERR_ARG;
    if (M == 0) return GPC_OK;
    const double dM = (double)M, dK = (double)K;
    Traced tr(h, GPC_K_OPS, dM * (dM + 1.0) * dK, 8.0 * (dM * dK + dM * dM));
    GemmArgs g{};
    g.M = M; g.N = M; g.K = K;
    g.A = A; g.lda = lda;
    g.B = A; g.ldb = lda;
    g.C = C; g.ldc = ldc;
    g.kchunk = K > 0 ? K : 1;
    GPC_HIP(h, gemm_f64(h->stream, TILE_128, false, true, EPI_SYMLOW, true, g, 1));
    return GPC_OK;
}

gpc_status gpc_multiply_transpose_adjoint(gpc_handle* h, int64_t M, int64_t K, const double* A, int64_t lda,
                                          const double* Cbar, int64_t ldcb, double beta, double* Abar, int64_t ldab)
{
    // C = A A^T:  Abar = (Cbar + Cbar^T) A + beta Abar
    if (!h || M < 0 || K < 0 || !(beta == 0.0 || beta == 1.0) || !ld_ok(K, lda) || !ld_ok(M, ldcb) ||
        !ld_ok(K, ldab) || (M > 0 && K > 0 && (!A || !Cbar || !Abar)))
        return GPC_ERR_ARG;
    if (overlap(Abar, M, K, ldab, A, M, K, lda) || overlap(Abar, M, K, ldab, Cbar, M, M, ldcb)) return GPC_ERR_ARG;
    if (M == 0 || K == 0) return GPC_OK;
    gpc_status st = gpc_gemm(h, 0, 0, M, K, M, Cbar, ldcb, A, lda, beta, Abar, ldab);
    if (st != GPC_OK) return st;
    return gpc_gemm(h, 1, 0, M, K, M, Cbar, ldcb, A, lda, 1.0, Abar, ldab);
}

gpc_status gpc_glm_bernoulli_logit(gpc_handle* h, int64_t n, int64_t k, const double* X, int64_t ldx,
                                   const int32_t* y, const double* alpha, const double* beta, double* lp,
                                   double* dalpha, double* dbeta, double* dX, int64_t lddx)
{
    if (!h || n < 0 || k < 0 || !ld_ok(k, ldx) || !alpha || !lp || !dalpha || (k > 0 && (!beta || !dbeta)) ||
        (n > 0 && (!y || (k > 0 && !X))) || (dX && !ld_ok(k, lddx)))
        return GPC_ERR_ARG;
    if (dX && (overlap(dX, n, k, lddx, X, n, k, ldx)))
        return GPC_ERR_ARG;
    gpc_status st = ensure_ws(h, sizeof(double) * (size_t)glm_workspace(n, k));
    if (st != GPC_OK) return st;
    const double dn = (double)n, dk = (double)k;
    Traced tr(h, GPC_K_OPS, 4.0 * dn * dk, 8.0 * dn * dk * (dX ? 2.0 : 1.0) + 4.0 * dn);
    GPC_HIP(h, glm_bernoulli_logit(h->stream, n, k, X, ldx, y, alpha, beta, lp, dalpha, dbeta, dX, lddx,
                                   (double*)h->ws));
    return GPC_OK;
}

gpc_status gpc_get_last_splits(const gpc_handle* h, int32_t* splits)
{
    if (!h || !splits) return GPC_ERR_ARG;
    *splits = h->last_splits;
    return GPC_OK;
}

}  // extern "C"
