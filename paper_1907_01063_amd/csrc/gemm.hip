// Tiled matrix products on the CDNA4 matrix cores (MFMA 16x16x4, FP64 or FP32).
//
// These are the dense contractions of the blocked Cholesky (the panel solve
// L21 = A21 L11^-T and the trailing update A22 - L21 L21^T of section 3.3.1)
// and of its blocked reverse sweep (the products of section 3.3.2).
//
// A workgroup owns a BM x BN output tile: 8 waves (2 x 4) for 128 x 128
// tiles, 4 waves (2 x 2) for 64 x 64; each wave owns a sub-tile made of 16x16
// MFMA blocks held in accumulator registers.  The k dimension is walked in chunks of BK: the next chunk is
// loaded from global memory into registers while the current chunk is consumed
// from LDS (two LDS buffers, one barrier per chunk).  Operands are staged in
// LDS k-major (sA[k][m], sB[k][n]) so that each MFMA operand fetch reads 16
// consecutive elements per k row.
//
// MFMA 16x16x4 register layout (one value per lane for A and B; 4 per lane
// for the 16x16 result): lane l supplies A[l%16][l/16] and B[l/16][l%16].
// The result rows differ by type (measured on gfx950): the FP64 instruction
// puts element (l/16 + 4r, l%16) in accumulator slot r, the FP32 instruction
// puts element (4*(l/16) + r, l%16) there.
#include <stdlib.h>

#include "gemm_tile.hpp"

namespace gpc {
namespace {

template <typename TI, int BM, int BN, int BK, int WM, int WN, bool AKM, bool BNK, int EPI, bool LOWER>
__global__ void __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(WM * WN == 8 ? 4 : 2)))
gemm_kernel(GemmArgs g)
{
    if (g.prio) __builtin_amdgcn_s_setprio(2);
    __shared__ TI lds[TileLds<TI, BM, BN, BK>::elems];
    // Workgroups are dealt to the 8 XCDs round-robin (dispatch id mod 8).
    // Renumber so that XCD x works on the x-th contiguous range of tiles:
    // consecutive tiles share their row panel, which then stays in that XCD's
    // L2.  A split-K launch (slices along z) renumbers its (slice, tile)
    // sequence as one, slice-major, so that an XCD takes whole slices and
    // reads each slice's operand chunks alone, instead of every XCD reading
    // the row panels of every slice.
    const bool flat = gridDim.z > 1 && gridDim.y == 1;
    const int nwg = flat ? gridDim.x * gridDim.z : gridDim.x;
    const int w = flat ? blockIdx.z * gridDim.x + blockIdx.x : blockIdx.x;
    const int u = xcd_item(w, nwg);
    const int t = flat ? u % (int)gridDim.x : u;
    const int z = flat ? u / (int)gridDim.x : (int)blockIdx.z;
    int64_t tm, tn;
    if (LOWER) {
        if (g.group > 1) grouped_lower_tile(t, (g.M + BM - 1) / BM, g.group, tm, tn);
        else lower_tile(t, tm, tn);
    } else {
        const int tilesN = (int)((g.N + BN - 1) / BN);
        if (g.group > 1) {
            grouped_tile(t, (g.M + BM - 1) / BM, tilesN, g.group, tm, tn);
        } else {
            tm = t / tilesN;
            tn = t % tilesN;
        }
    }
    // tile coordinates are uniform: keep them (and all that derives from
    // them) in scalar registers
    tm = __builtin_amdgcn_readfirstlane((int)tm);
    tn = __builtin_amdgcn_readfirstlane((int)tn);
    // member blockIdx.y of a batch of equal-shape products (0 when unbatched)
    GemmArgs gb = g;
    gb.A = (const TI*)g.A + blockIdx.y * g.bsA;
    gb.B = (const TI*)g.B + blockIdx.y * g.bsB;
    gb.C = g.C + blockIdx.y * g.bsC;
    gemm_tile<TI, BM, BN, BK, WM, WN, AKM, BNK, EPI, LOWER>(gb, tm, tn, __builtin_amdgcn_readfirstlane(z), lds);
}

// Row panels kept per XCD by the grouped tile order: as many BM-row panels
// of the launch's k-chunk as fit in `group_bytes` (at most 16).  The budget
// is half of an XCD's 4 MiB L2 by default; the environment variable
// GPC_TILE_GROUP_KIB sets it (0 = row-by-row order), read once per process.
int64_t group_bytes()
{
    static const int64_t v = [] {
        const char* e = getenv("GPC_TILE_GROUP_KIB");
        return e ? (int64_t)atoll(e) * 1024 : (int64_t)2048 * 1024;
    }();
    return v;
}

// A product of at most 16 tile rows and more than 8 tile columns walks its
// tiles column by column (one band of all its rows): the tile rows of one
// column, which share its column panel, then run together on one XCD, so
// each column panel is read about once instead of once per tile row (each
// XCD reads the few row panels, the larger operand once).
template <typename TI, int BM, int BN, bool LOWER>
int tile_group(const GemmArgs& g)
{
    const int64_t tilesM = (g.M + BM - 1) / BM, tilesN = (g.N + BN - 1) / BN;
    if (!LOWER && group_bytes() > 0 && tilesM > 1 && tilesM <= 16 && tilesN > 8) return (int)tilesM;
    const int64_t kc = g.kchunk < g.K ? g.kchunk : g.K;
    const int64_t panel = (int64_t)BM * (kc > 0 ? kc : 1) * (int64_t)sizeof(TI);
    const int64_t G = group_bytes() / panel;
    return (int)(G < 2 ? 1 : G > 16 ? 16 : G);
}

template <typename TI, int BM, int BN, int BK, int WM, int WN, bool AKM, bool BNK, int EPI, bool LOWER>
hipError_t launch(hipStream_t s, const GemmArgs& g, int splits, int batch)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    int64_t tiles;
    if (LOWER) {
        const int64_t t = (g.M + BM - 1) / BM;
        tiles = t * (t + 1) / 2;
    } else {
        tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    }
    dim3 grid((unsigned)tiles, (unsigned)(batch < 1 ? 1 : batch), (unsigned)(splits < 1 ? 1 : splits));
    GemmArgs ga = g;
    ga.group = tile_group<TI, BM, BN, LOWER>(g);
    hipLaunchKernelGGL((gemm_kernel<TI, BM, BN, BK, WM, WN, AKM, BNK, EPI, LOWER>), grid, dim3(WM * WN * 64), 0, s, ga);
    return hipGetLastError();
}

// The tile loads (operands, and C for the subtracting products) use 32-bit
// byte offsets within a 128-row (or k-row) band.
bool ld_fits(const GemmArgs& g)
{
    return g.lda <= (int64_t(1) << 20) && g.ldb <= (int64_t(1) << 20) && g.ldah <= (int64_t(1) << 20) &&
           g.ldc <= (int64_t(1) << 20);
}

}  // namespace

#define GPC_GEMM_CASE(TI, CFG, BM, BN, BK, AKM, BNK, EPI, LOWER)                                 \
    if (cfg == CFG && a_km == AKM && b_nk == BNK && epi == EPI && lower_tiles == LOWER)           \
        return launch<TI, BM, BN, BK, 2, (BN == 128 ? 4 : 2), AKM, BNK, EPI, LOWER>(s, g, splits, batch);

hipError_t gemm_f64(hipStream_t s, TileCfg cfg, bool a_km, bool b_nk, Epi epi, bool lower_tiles,
                    const GemmArgs& g, int splits, int batch)
{
    if (!ld_fits(g)) return hipErrorInvalidValue;
    // trailing narrow update (C strict upper masked at run time)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, true, EPI_SUB, false)
    // trailing SYRK (lower tiles), panel solve, adjoint panel solve and updates
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, true, EPI_SUB, true)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, true, EPI_STORE, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, false, EPI_STORE, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, false, EPI_SUB, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, true, false, EPI_PARTIAL, false)
    GPC_GEMM_CASE(double, TILE_64, 64, 64, 16, true, false, EPI_PARTIAL, false)
    // panel solves with twice the workgroups (64-row tiles spanning all N).
    // The reverse sweep's (B stored K x N) takes k-chunks of 32: its 100 KB of
    // LDS keep its workgroups off CUs that the side stream's products hold,
    // which pace the sweep
    GPC_GEMM_CASE(double, TILE_64W, 64, 128, 16, false, true, EPI_STORE, false)
    GPC_GEMM_CASE(double, TILE_64W, 64, 128, 32, false, false, EPI_STORE, false)
    // skinny narrow update (more, smaller tiles)
    GPC_GEMM_CASE(double, TILE_64, 64, 64, 16, false, true, EPI_SUB, false)
    // diagonal-block reverse step
    GPC_GEMM_CASE(double, TILE_64, 64, 64, 16, true, false, EPI_SYMLOW, false)
    GPC_GEMM_CASE(double, TILE_64, 64, 64, 16, false, false, EPI_STORE, false)
    GPC_GEMM_CASE(double, TILE_64, 64, 64, 16, true, false, EPI_PHI, false)
    // general products op(A) op(B) (section 3.1) and their split-K slices;
    // lower-tile products for the reverse modes of the triangular solve and
    // inverse, and C = A A^T mirrored over the diagonal
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, true, false, EPI_STORE, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, true, true, EPI_STORE, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, false, EPI_ADD, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, true, EPI_ADD, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, true, false, EPI_ADD, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, true, true, EPI_ADD, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, false, EPI_PARTIAL, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, true, EPI_PARTIAL, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, true, true, EPI_PARTIAL, false)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, true, EPI_STORE, true)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, true, true, EPI_STORE, true)
    GPC_GEMM_CASE(double, TILE_128, 128, 128, 16, false, true, EPI_SYMLOW, true)
    return hipErrorInvalidValue;
}

hipError_t gemm_f32in(hipStream_t s, TileCfg cfg, bool a_km, bool b_nk, Epi epi, bool lower_tiles,
                      const GemmArgs& g, int splits, int batch)
{
    if (!ld_fits(g)) return hipErrorInvalidValue;
    GPC_GEMM_CASE(float, TILE_128, 128, 128, 32, false, true, EPI_SUB, false)
    GPC_GEMM_CASE(float, TILE_128, 128, 128, 32, false, true, EPI_SUB, true)
    GPC_GEMM_CASE(float, TILE_128, 128, 128, 32, false, false, EPI_SUB, false)
    GPC_GEMM_CASE(float, TILE_128, 128, 128, 32, true, false, EPI_PARTIAL, false)
    GPC_GEMM_CASE(float, TILE_64, 64, 64, 32, true, false, EPI_PARTIAL, false)
    GPC_GEMM_CASE(float, TILE_64, 64, 64, 32, false, true, EPI_SUB, false)
    return hipErrorInvalidValue;
}

}  // namespace gpc
