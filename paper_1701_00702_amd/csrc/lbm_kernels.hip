// Kernels for the enthalpy-based MRT lattice Boltzmann method for
// solid-liquid phase change in metal foams under local thermal
// non-equilibrium (Liu, He & Li, arXiv:1701.00702), written for gfx950.
//
// One launch of step_kernel advances every node of every cavity by one time
// step.  One thread per node, pull streaming, structure-of-arrays planes,
// A/B buffers; per node (lbm_node.h):
//   1. pull the post-collision populations of the neighbours (Eqs. 15, 33,
//      44; 27 with D2Q9 thermal fields, 19 with the D2Q5 ones of Appendix B);
//      a wall node instead pulls the populations of its interior partner
//      and rebuilds its own by non-equilibrium extrapolation (Eq. 52 and its
//      thermal analogues);
//   2. H (Eq. 37), T_f and f_l without iteration (Eqs. 38-39), T_m (Eq. 48),
//      rho (Eq. 21), the volumetric blend with the solid at rest (Eq. 20),
//      buoyancy (Eq. 7), explicit velocity (Eqs. 23-25), total force (Eq. 3);
//   3. the flow collision in moment space with forcing (Eqs. 14, 16-19);
//   4. interstitial sources with the backward-difference time derivative
//      (Eqs. 36, 47, Remark III);
//   5. the enthalpy and metal-foam collisions (Eqs. 32, 34-35; 43, 45-46;
//      Eqs. B1-B5 on D2Q5);
//   6. store the post-collision populations and the source, and tally the
//      energy/mass carried across wall links (FP64, one slot per
//      wall-adjacent node, no atomics).
// The 9x9 transforms are expanded by hand (entries 0, +-1, +-2, +-4) and the
// work stays on the vector ALUs: at about two flops per byte the step is
// bound by HBM bandwidth, not by matrix throughput.

#include "lbm_node.h"
#include "lbm_tiles.h"

namespace lbm {

int bytes_per_node(int storage) {
    switch (storage) {
        case ST_F64: return LayoutOf<ST_F64>::L::bytes_per_node;
        case ST_F32: return LayoutOf<ST_F32>::L::bytes_per_node;
        case ST_F16: return LayoutOf<ST_F16>::L::bytes_per_node;
        case ST_BF16: return LayoutOf<ST_BF16>::L::bytes_per_node;
        case ST_F16S: return LayoutOf<ST_F16S>::L::bytes_per_node;
        case ST_BF16S: return LayoutOf<ST_BF16S>::L::bytes_per_node;
        case ST_F32H: return LayoutOf<ST_F32H>::L::bytes_per_node;
        case ST5_F64: return LayoutOf<ST5_F64>::L::bytes_per_node;
        case ST5_F32: return LayoutOf<ST5_F32>::L::bytes_per_node;
        case ST5_F32H: return LayoutOf<ST5_F32H>::L::bytes_per_node;
    }
    return 0;
}

// Dispatch a templated launcher on the storage form.
#define LBM_DISPATCH(storage, FN, ...)                                     \
    switch (storage) {                                                     \
        case ST_F64: return FN<ST_F64>(__VA_ARGS__);                       \
        case ST_F32: return FN<ST_F32>(__VA_ARGS__);                       \
        case ST_F16: return FN<ST_F16>(__VA_ARGS__);                       \
        case ST_BF16: return FN<ST_BF16>(__VA_ARGS__);                     \
        case ST_F16S: return FN<ST_F16S>(__VA_ARGS__);                     \
        case ST_BF16S: return FN<ST_BF16S>(__VA_ARGS__);                   \
        case ST_F32H: return FN<ST_F32H>(__VA_ARGS__);                     \
        case ST5_F64: return FN<ST5_F64>(__VA_ARGS__);                     \
        case ST5_F32: return FN<ST5_F32>(__VA_ARGS__);                     \
        case ST5_F32H: return FN<ST5_F32H>(__VA_ARGS__);                   \
        default: return hipErrorInvalidValue;                              \
    }

// ---------------------------------------------------------------------------
// The fused step kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int remap_block(int b, int grid, int xcd_remap) {
    // Hardware hands consecutive workgroups to the 8 XCDs in turn; this maps
    // them back so that each XCD walks a contiguous range of tiles.
    if (!xcd_remap) return b;
    const int full = grid & ~7;
    if (b >= full) return b;
    const int per = full >> 3;
    return (b & 7) * per + (b >> 3);
}

// The tile of one workgroup.  Accesses are 32-bit offsets from the block of
// the band of a row the workgroup shares: for interior tiles the row before
// their first one (the pulls reach one row either side; a tile of at most
// 2048 pitched nodes then spans at most 2048 / nx + 3 rows, so two bands),
// for wall tiles (one row each) the first of the three rows their wall
// partners pull from.  Both kinds share one instantiation of the node
// update (decided per node), so the kernel holds a single copy of the
// global accesses.
template <class Lay, typename R, typename RH, bool PULL, int NPT>
__device__ __forceinline__ void step_tile(const void *__restrict__ src, void *__restrict__ dst,
                                          const R *__restrict__ sr_src, R *__restrict__ sr_dst,
                                          double *__restrict__ acc, const CavityConst<R> *__restrict__ cav,
                                          const Tile &tl) {
    const CavityConst<R> &c = cav[tl.cav];
    const bool wall = tl.kind != TILE_INTERIOR;
    int yb;
    if (wall) {
        yb = tl.k0 < c.nx ? 0 : c.ny - 3;
    } else {
        const int y0 = tl.k0 / c.pitch;
        yb = y0 >= 1 ? y0 - 1 : 0;
    }
    const BandOrigin org = band_origin(c, yb);
    const int ba = yb / c.band_rows;
    const void *sblk = band_block(c, src, ba);
    void *dblk = band_block(c, dst, ba);
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int k = tl.k0 + (int)threadIdx.x + j * (int)blockDim.x;
        if (k < tl.k1) {
            int x, y;
            if (wall) {
                ring_node(c, k, x, y);
            } else {
                y = k / c.pitch;
                x = k - y * c.pitch;
            }
            // interior tiles cover whole (pitched) rows: the wall columns ride
            // along (each stored cache line then has one writer); lanes on
            // the row padding idle
            if (wall || x < c.nx)
                step_node_at<Lay, R, RH, PULL>(c, sblk, dblk, sr_src, sr_dst, acc, x, y, org);
        }
    }
}

// One tile per workgroup, or (LOOP) a grid-stride walk over the tiles for
// the persistent launch.
template <class Lay, typename R, typename RH, bool PULL, int NPT, bool LOOP>
__global__ __launch_bounds__(512) void step_kernel(const void *__restrict__ src, void *__restrict__ dst,
                                                   const R *__restrict__ sr_src,
                                                   R *__restrict__ sr_dst, double *__restrict__ acc,
                                                   const CavityConst<R> *__restrict__ cav,
                                                   const Tile *__restrict__ tiles, int ntiles,
                                                   int xcd_remap) {
    const int b = remap_block(blockIdx.x, gridDim.x, xcd_remap);
    if (!LOOP) {
        if (b < ntiles) step_tile<Lay, R, RH, PULL, NPT>(src, dst, sr_src, sr_dst, acc, cav, tiles[b]);
        return;
    }
    for (int t = b; t < ntiles; t += gridDim.x)
        step_tile<Lay, R, RH, PULL, NPT>(src, dst, sr_src, sr_dst, acc, cav, tiles[t]);
}

template <int ST, bool PULL, int NPT>
static hipError_t launch_step_t(const StepLaunch &L, hipStream_t s) {
    using Lay = typename LayoutOf<ST>::L;
    using R = typename LayoutOf<ST>::R;
    using RH = typename LayoutOf<ST>::RH;
    if (L.grid >= L.ntiles)
        hipLaunchKernelGGL((step_kernel<Lay, R, RH, PULL, NPT, false>), dim3(L.grid), dim3(L.block), 0, s, L.src,
                           L.dst, (const R *)L.sr_src, (R *)L.sr_dst, L.acc,
                           (const CavityConst<R> *)L.cav, L.tiles, L.ntiles, L.xcd_remap);
    else
        hipLaunchKernelGGL((step_kernel<Lay, R, RH, PULL, NPT, true>), dim3(L.grid), dim3(L.block), 0, s, L.src,
                           L.dst, (const R *)L.sr_src, (R *)L.sr_dst, L.acc,
                           (const CavityConst<R> *)L.cav, L.tiles, L.ntiles, L.xcd_remap);
    return hipGetLastError();
}

template <int ST, bool PULL>
static hipError_t launch_step_p(const StepLaunch &L, hipStream_t s) {
    // the tile width is block * npt, so every variant must use the same npt
    switch (L.npt) {
        case 1: return launch_step_t<ST, PULL, 1>(L, s);
        case 2: return launch_step_t<ST, PULL, 2>(L, s);
        case 4: return launch_step_t<ST, PULL, 4>(L, s);
        default: return hipErrorInvalidValue;
    }
}

template <int ST>
static hipError_t launch_step_s(const StepLaunch &L, hipStream_t s) {
    return L.pull ? launch_step_p<ST, true>(L, s) : launch_step_p<ST, false>(L, s);
}

hipError_t launch_step(const StepLaunch &L, hipStream_t s) {
    if (L.block < 64 || L.block > 512 || (L.block & 63) || L.grid < 1 || L.ntiles < 1)
        return hipErrorInvalidValue;
    LBM_DISPATCH(L.storage, launch_step_s, L, s)
}

// ---------------------------------------------------------------------------
// K steps per launch through LDS (K = 2, 3).  One workgroup per tile: the
// first update covers the tile and its (K-1)-node ring into LDS, a middle
// update (K = 3) the tile and a one-node ring in place in LDS, the last
// update the tile into the destination buffer, with barriers between.  Tile
// shapes fill at most 64 KiB of LDS; the defaults (measured) let three or
// four workgroups share a CU, whose waves overlap one tile's loads with
// another's arithmetic.  Two-step tiles first.
// ---------------------------------------------------------------------------
// One tile per workgroup, or (LOOP) a grid-stride walk over the tiles for
// the persistent launch.  Without the loop nothing in the tile's code is
// loop-invariant, so the compiler does not keep the 27 plane addresses live
// across iterations (they would spill to vector registers).
template <class Lay, typename R, typename RH, int TW, int TH, int NT, int K>
__device__ __forceinline__ void stepk_advance(const void *__restrict__ src, void *__restrict__ dst,
                                              const R *__restrict__ sr_src, R *__restrict__ sr_dst,
                                              double *__restrict__ acc, const CavityConst<R> *__restrict__ cav,
                                              const Tile2 &tl, void *lds_q, R *lds_sr, float *lds_b) {
    using Sh = StepKShape<Lay, TW, TH, K>;
    const CavityConst<R> &c = cav[tl.cav];
    // NT >= NFIRST: each thread advances at most one node per update
    const int s = (int)threadIdx.x;
    if constexpr (Sh::STAGE_BASE) {
        stepk_stage_bases<Lay, R, TW, TH, K, NT>(c, tl, src, lds_b, s);
        __syncthreads();
    }
    if (s < Sh::LW * (tl.h + 2 * Sh::RING))
        stepk_first<Lay, R, RH, TW, TH, K>(c, tl, src, sr_src, acc, lds_q, lds_sr, lds_b, s);
    __syncthreads();
#pragma unroll
    for (int j = K - 2; j >= 1; --j) {
        MidNode<R, RH> n;
        const bool act = s < (TW + 2 * j) * (tl.h + 2 * j) &&
                         stepk_mid_load<Lay, R, RH, TW, TH, K>(c, tl, j, lds_q, lds_sr, s, n);
        __syncthreads();  // every pull of this update is in registers
        if (act) stepk_mid_store<Lay, R, RH, TW, TH, K>(c, tl, acc, lds_q, lds_sr, n);
        __syncthreads();
    }
    if (s < TW * tl.h) stepk_last<Lay, R, RH, TW, TH, K>(c, tl, dst, sr_dst, acc, lds_q, lds_sr, s);
}

// Waves per SIMD a multi-step kernel is built for: as many workgroups per
// CU as the LDS of one tile allows (160 KiB per CU; at most 32 waves per
// CU), so that the register budget never holds residency below that.
template <class Lay, typename R, int TW, int TH, int NT, int K>
constexpr int stepk_waves_per_eu() {
    using Sh = StepKShape<Lay, TW, TH, K>;
    constexpr int lds = (int)(Sh::LDS_BYTES + Sh::NSLOT * sizeof(R) + Sh::BASE_BYTES);
    constexpr int by_lds = (160 * 1024) / lds;
    constexpr int by_waves = 32 / (NT / 64);
    constexpr int wgs = by_lds < by_waves ? by_lds : by_waves;
    return (wgs * (NT / 64) + 3) / 4;
}

// Storage forms whose single-tile multi-step kernels carry that occupancy
// as a waves-per-EU bound (bit ST of the mask).  Measured on the 8192^2
// cavity: the FP32 D2Q5 forms keep their registers (50 and 57) and gain
// 5% (three steps) and 3-4% (two steps) from the schedule the bound
// selects; FP32 D2Q9 is unchanged (LDS holds it at three workgroups per
// CU); the 16-bit and D2Q9 FP32_H64 forms fit the bound only by spilling
// and lose 5-24%.
#ifndef LBM_WPE_MASK
#define LBM_WPE_MASK ((1 << ST5_F32) | (1 << ST5_F32H))
#endif
template <int ST, class Lay, typename R, int TW, int TH, int NT, int K>
constexpr int stepk_wpe() {
    return ((LBM_WPE_MASK >> ST) & 1) ? stepk_waves_per_eu<Lay, R, TW, TH, NT, K>() : 1;
}

template <class Lay, typename R, typename RH, int TW, int TH, int NT, int K, bool LOOP, int WPE>
__global__ __launch_bounds__(NT, WPE) void stepk_kernel(const void *__restrict__ src, void *__restrict__ dst,
                                                   const R *__restrict__ sr_src,
                                                   R *__restrict__ sr_dst, double *__restrict__ acc,
                                                   const CavityConst<R> *__restrict__ cav,
                                                   const Tile2 *__restrict__ tiles, int ntiles, int xcd_remap) {
    using Sh = StepKShape<Lay, TW, TH, K>;
    static_assert(Sh::LDS_BYTES + Sh::NSLOT * sizeof(R) + Sh::BASE_BYTES <= 65536, "tile exceeds 64 KiB of LDS");
    static_assert(NT >= Sh::NFIRST && NT % 64 == 0, "one thread per node of the first update");
    __shared__ __align__(16) unsigned char lds_q[Sh::LDS_BYTES];
    __shared__ R lds_sr[Sh::NSLOT];
    __shared__ float lds_b[Sh::STAGE_BASE ? 3 * Sh::NBASE : 1];
    const int b = remap_block(blockIdx.x, gridDim.x, xcd_remap);
    if (!LOOP) {
        if (b < ntiles)
            stepk_advance<Lay, R, RH, TW, TH, NT, K>(src, dst, sr_src, sr_dst, acc, cav, tiles[b], lds_q, lds_sr,
                                                     lds_b);
        return;
    }
    for (int t = b; t < ntiles; t += gridDim.x) {
        stepk_advance<Lay, R, RH, TW, TH, NT, K>(src, dst, sr_src, sr_dst, acc, cav, tiles[t], lds_q, lds_sr, lds_b);
        __syncthreads();  // the next tile reuses the LDS
    }
}

template <int ST, int K, int I>
static hipError_t launch_stepk_i(const Step2Launch &L, hipStream_t s) {
    using Lay = typename LayoutOf<ST>::L;
    using R = typename LayoutOf<ST>::R;
    using RH = typename LayoutOf<ST>::RH;
    using Tl = StepKTileI<ST, K, I>;
    if (L.grid >= L.ntiles) {
        hipLaunchKernelGGL((stepk_kernel<Lay, R, RH, Tl::TW, Tl::TH, Tl::NT, K, false,
                                         stepk_wpe<ST, Lay, R, Tl::TW, Tl::TH, Tl::NT, K>()>),
                           dim3(L.grid), dim3(Tl::NT),
                           0, s, L.src, L.dst, (const R *)L.sr_src, (R *)L.sr_dst, L.acc,
                           (const CavityConst<R> *)L.cav, L.tiles, L.ntiles, L.xcd_remap);
    } else {
        // persistent grids exist for the default shape only
        if constexpr (I == 0)
            hipLaunchKernelGGL((stepk_kernel<Lay, R, RH, Tl::TW, Tl::TH, Tl::NT, K, true, 1>), dim3(L.grid),
                               dim3(Tl::NT), 0, s, L.src, L.dst, (const R *)L.sr_src, (R *)L.sr_dst, L.acc,
                               (const CavityConst<R> *)L.cav, L.tiles, L.ntiles, L.xcd_remap);
        else
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int ST, int K>
static hipError_t launch_stepk_s(const Step2Launch &L, hipStream_t s) {
    switch (L.shape) {
        case 0: return launch_stepk_i<ST, K, 0>(L, s);
        case 1: return launch_stepk_i<ST, K, 1>(L, s);
        case 2: return launch_stepk_i<ST, K, 2>(L, s);
        default: return hipErrorInvalidValue;
    }
}

bool stepk_supported(int storage, int k) { return stepk_available(storage, k); }

template <int ST, int K>
static void tile_of(int shape, int *tw, int *th) {
    const TileDims d = dims_of<ST, K>(shape);
    *tw = d.tw;
    *th = d.th;
}

void stepk_tile(int storage, int k, int shape, int *tw, int *th) {
    *tw = *th = 0;
    if (shape < 0 || shape >= kTileShapes) return;
    if (k == 3) {
        switch (storage) {
            case ST_F32: return tile_of<ST_F32, 3>(shape, tw, th);
            case ST5_F32: return tile_of<ST5_F32, 3>(shape, tw, th);
            case ST_F32H: return tile_of<ST_F32H, 3>(shape, tw, th);
            case ST5_F32H: return tile_of<ST5_F32H, 3>(shape, tw, th);
            case ST_F16: return tile_of<ST_F16, 3>(shape, tw, th);
            case ST_BF16: return tile_of<ST_BF16, 3>(shape, tw, th);
            case ST_F16S: return tile_of<ST_F16S, 3>(shape, tw, th);
            case ST_BF16S: return tile_of<ST_BF16S, 3>(shape, tw, th);
            default: return;
        }
    }
    if (k != 2) return;
    switch (storage) {
        case ST_F16: return tile_of<ST_F16, 2>(shape, tw, th);
        case ST_BF16: return tile_of<ST_BF16, 2>(shape, tw, th);
        case ST_F16S: return tile_of<ST_F16S, 2>(shape, tw, th);
        case ST_BF16S: return tile_of<ST_BF16S, 2>(shape, tw, th);
        case ST_F32: return tile_of<ST_F32, 2>(shape, tw, th);
        case ST5_F32: return tile_of<ST5_F32, 2>(shape, tw, th);
        case ST_F64: return tile_of<ST_F64, 2>(shape, tw, th);
        case ST5_F64: return tile_of<ST5_F64, 2>(shape, tw, th);
        case ST_F32H: return tile_of<ST_F32H, 2>(shape, tw, th);
        case ST5_F32H: return tile_of<ST5_F32H, 2>(shape, tw, th);
        default: return;
    }
}

hipError_t launch_stepk(const Step2Launch &L, hipStream_t s) {
    if (L.grid < 1 || L.ntiles < 1) return hipErrorInvalidValue;
    if (L.steps == 3) {
        switch (L.storage) {
            case ST_F32: return launch_stepk_s<ST_F32, 3>(L, s);
            case ST5_F32: return launch_stepk_s<ST5_F32, 3>(L, s);
            case ST_F32H: return launch_stepk_s<ST_F32H, 3>(L, s);
            case ST5_F32H: return launch_stepk_s<ST5_F32H, 3>(L, s);
            case ST_F16: return launch_stepk_s<ST_F16, 3>(L, s);
            case ST_BF16: return launch_stepk_s<ST_BF16, 3>(L, s);
            case ST_F16S: return launch_stepk_s<ST_F16S, 3>(L, s);
            case ST_BF16S: return launch_stepk_s<ST_BF16S, 3>(L, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (L.steps != 2) return hipErrorInvalidValue;
    switch (L.storage) {
        case ST_F32: return launch_stepk_s<ST_F32, 2>(L, s);
        case ST5_F32: return launch_stepk_s<ST5_F32, 2>(L, s);
        case ST_F64: return launch_stepk_s<ST_F64, 2>(L, s);
        case ST5_F64: return launch_stepk_s<ST5_F64, 2>(L, s);
        case ST_F32H: return launch_stepk_s<ST_F32H, 2>(L, s);
        case ST5_F32H: return launch_stepk_s<ST5_F32H, 2>(L, s);
        case ST_F16: return launch_stepk_s<ST_F16, 2>(L, s);
        case ST_BF16: return launch_stepk_s<ST_BF16, 2>(L, s);
        case ST_F16S: return launch_stepk_s<ST_F16S, 2>(L, s);
        case ST_BF16S: return launch_stepk_s<ST_BF16S, 2>(L, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Macroscopic fields of a range of rows of one cavity, and the reductions of
// the diagnostics.
// ---------------------------------------------------------------------------
constexpr int MB = 256;  // threads per block of the diagnostics kernels

// Workgroups covering rows nodes of a row range, one node per thread.
static int row_blocks(int nx, int rows) { return (int)(((int64_t)nx * rows + MB - 1) / MB); }

// Block reduction of N doubles per thread (maxima for P_DT and P_U, sums
// otherwise), in a fixed order, so the diagnostics are deterministic: a
// butterfly across each 64-lane wavefront (after it every lane holds the
// same value, the operations being commutative), then the MB / 64 wave
// results in wave order.  The result is valid in thread 0.
template <int N>
__device__ __forceinline__ void block_reduce(double v[N], double (*sh)[MB / 64]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double o = __shfl_xor(v[k], off, 64);
            v[k] = (k == P_DT || k == P_U) ? fmax(v[k], o) : v[k] + o;
        }
    }
    const int w = (int)threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) sh[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double a = sh[k][0];
            for (int q = 1; q < MB / 64; ++q) a = (k == P_DT || k == P_U) ? fmax(a, sh[k][q]) : a + sh[k][q];
            v[k] = a;
        }
    }
}

template <class Lay, typename R, typename RH>
__global__ __launch_bounds__(MB) void macro_kernel(const void *__restrict__ src,
                                                   const CavityConst<R> *__restrict__ cav, int ci,
                                                   int raw, int y0, int rows, double *__restrict__ fields) {
    const CavityConst<R> &c = cav[ci];
    const int nx = c.nx;
    const int64_t nn = (int64_t)nx * rows;
    const int64_t kk = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (kk >= nn) return;
    double out[6], v[NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k) v[k] = 0.0;
    macro_node<Lay, R, RH>(c, src, raw != 0, (int)(kk % nx), y0 + (int)(kk / nx), out, v);
#pragma unroll
    for (int q = 0; q < 6; ++q) fields[q * nn + kk] = out[q];
}

template <int ST>
static hipError_t launch_macro_s(const MacroLaunch &L, int nx, hipStream_t s) {
    using Lay = typename LayoutOf<ST>::L;
    using R = typename LayoutOf<ST>::R;
    using RH = typename LayoutOf<ST>::RH;
    hipLaunchKernelGGL((macro_kernel<Lay, R, RH>), dim3(row_blocks(nx, L.rows)), dim3(MB), 0, s, L.src,
                       (const CavityConst<R> *)L.cav, L.cav_index, L.raw, L.y0, L.rows, L.fields);
    return hipGetLastError();
}

hipError_t launch_macro(const MacroLaunch &L, int nx, int ny, hipStream_t s) {
    if (L.y0 < 0 || L.rows < 1 || L.rows > ny - L.y0) return hipErrorInvalidValue;
    LBM_DISPATCH(L.storage, launch_macro_s, L, nx, s)
}

// Final pass: fixed-order sums of the block partials, Nusselt numbers from
// one-sided second-order differences, the melt front on the middle row and
// the wall tallies.
__global__ __launch_bounds__(MB) void diag_kernel(DiagLaunch L) {
    const int t = threadIdx.x;
    const int nx = L.nx, ny = L.ny;
    __shared__ double sh[NPART + 3 + 8][MB / 64];
    double v[NPART + 3 + 8];
#pragma unroll
    for (int k = 0; k < NPART + 11; ++k) v[k] = 0.0;
    for (int b = t; b < L.nblocks; b += MB) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) {
            const double a = L.partials[(int64_t)b * NPART + k];
            v[k] = (k == P_DT || k == P_U) ? fmax(v[k], a) : v[k] + a;
        }
    }
    if (!L.periodic) {
        for (int y = 1 + t; y <= ny - 2; y += MB) {
            const double *Tf = L.tf + (int64_t)y * 6;
            const double *Tm = L.tm + (int64_t)y * 6;
            const double dTf = (-3.0 * Tf[0] + 4.0 * Tf[1] - Tf[2]) * 0.5;
            const double dTm = (-3.0 * Tm[0] + 4.0 * Tm[1] - Tm[2]) * 0.5;
            v[NPART + 0] += dTf;  // PCM-only gradient
            const double cTf = (3.0 * Tf[5] - 4.0 * Tf[4] + Tf[3]) * 0.5;
            const double cTm = (3.0 * Tm[5] - 4.0 * Tm[4] + Tm[3]) * 0.5;
            v[NPART + 1] += L.kf * dTf + L.km * dTm;
            v[NPART + 2] += L.kf * cTf + L.km * cTm;
        }
    }
    // wall tallies: slots [left ny][right ny][bottom nx][top nx]
    const double *acc = L.acc + 2 * L.acc0;
    for (int y = t; y < ny; y += MB) {
        v[NPART + 3] += acc[2 * y];
        v[NPART + 4] += acc[2 * (ny + y)];
        v[NPART + 7] += acc[2 * y + 1];
        v[NPART + 8] += acc[2 * (ny + y) + 1];
    }
    for (int x = t; x < nx; x += MB) {
        v[NPART + 5] += acc[2 * (2 * ny + x)];
        v[NPART + 6] += acc[2 * (2 * ny + nx + x)];
        v[NPART + 9] += acc[2 * (2 * ny + x) + 1];
        v[NPART + 10] += acc[2 * (2 * ny + nx + x) + 1];
    }
    block_reduce<NPART + 11>(v, sh);
    if (t == 0) {
        double *o = L.out;
        const double nint = L.periodic ? (double)nx * (ny - 2) : (double)(nx - 2) * (ny - 2);
        o[D_FL] = v[P_FL] / nint;
        o[D_E] = v[P_E];
        o[D_M] = v[P_M];
        o[D_DT] = v[P_DT];
        o[D_U] = v[P_U];
        o[D_NF] = v[P_NF];
        const double nrow = (double)(ny - 2);
        o[D_NUH] = L.periodic ? 0.0 : -(L.L / (L.ke * L.dT)) * (v[NPART + 1] / nrow);
        o[D_NUHP] = L.periodic ? 0.0 : -(L.L / L.dT) * (v[NPART + 0] / nrow);
        o[D_NUC] = L.periodic ? 0.0 : -(L.L / (L.ke * L.dT)) * (v[NPART + 2] / nrow);
        // melt front: first f_l = 0.5 crossing on row ny/2 seen from x = 0
        double xf = 1.0;
        if (!L.periodic) {
            const double *fl = L.fl_mid;
            if (fl[0] < 0.5) {
                xf = 0.0;
            } else {
                for (int i = 0; i + 1 < nx; ++i) {
                    const double a = fl[i], b = fl[i + 1];
                    if (a >= 0.5 && b < 0.5) {
                        xf = (i + (a - 0.5) / (a - b)) / L.L;
                        break;
                    }
                }
            }
        } else {
            xf = 0.0;
        }
        o[D_FRONT] = xf;
        for (int w = 0; w < 4; ++w) {
            o[D_FLUXE + w] = v[NPART + 3 + w] + v[P_INE0 + w];
            o[D_FLUXM + w] = v[NPART + 7 + w] + v[P_INM0 + w];
        }
    }
}

hipError_t launch_diag(const DiagLaunch &L, int nx, int ny, hipStream_t s) {
    if (L.nx != nx || L.ny != ny) return hipErrorInvalidValue;
    hipLaunchKernelGGL(diag_kernel, dim3(1), dim3(MB), 0, s, L);
    return hipGetLastError();
}

// The per-node part of the diagnostics, without field planes: a fixed grid
// strides over the cavity's nodes; each thread folds its nodes'
// contributions (macro_node's per-node values) in node order, then a
// fixed-order block reduction gives one partial per workgroup.  The
// temperatures of the three columns next to each vertical wall and the
// middle row's liquid fraction go to compact arrays (tf/tm: [ny][6], column
// k for x = 0, 1, 2, nx - 3, nx - 2, nx - 1; fl_mid: [nx]).  Every element
// of the partials and of the compact arrays is written, so nothing needs
// clearing beforehand.
int diag_node_blocks(int nx, int ny) {
    const int64_t b = ((int64_t)nx * ny + MB - 1) / MB;
    return (int)(b < LBM_DIAG_MAX_BLOCKS ? b : LBM_DIAG_MAX_BLOCKS);
}

template <class Lay, typename R, typename RH>
__global__ __launch_bounds__(MB) void diag_node_kernel(const void *__restrict__ src,
                                                       const CavityConst<R> *__restrict__ cav, int ci, int raw,
                                                       double *__restrict__ partials, double *__restrict__ tf,
                                                       double *__restrict__ tm, double *__restrict__ fl_mid) {
    const CavityConst<R> &c = cav[ci];
    const int nx = c.nx, ny = c.ny;
    const int64_t nn = (int64_t)nx * ny;
    double tot[NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k) tot[k] = 0.0;
    for (int64_t kk = (int64_t)blockIdx.x * MB + threadIdx.x; kk < nn; kk += (int64_t)gridDim.x * MB) {
        const int x = (int)(kk % nx), y = (int)(kk / nx);
        double out[6], v[NPART];
#pragma unroll
        for (int k = 0; k < NPART; ++k) v[k] = 0.0;
        macro_node<Lay, R, RH>(c, src, raw != 0, x, y, out, v);
#pragma unroll
        for (int k = 0; k < NPART; ++k) tot[k] = (k == P_DT || k == P_U) ? fmax(tot[k], v[k]) : tot[k] + v[k];
        const int cols[6] = {0, 1, 2, nx - 3, nx - 2, nx - 1};
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (x == cols[k]) {
                tf[(int64_t)y * 6 + k] = out[2];
                tm[(int64_t)y * 6 + k] = out[3];
            }
        if (y == ny / 2) fl_mid[x] = out[4];
    }
    __shared__ double sh[NPART][MB / 64];
    block_reduce<NPART>(tot, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) partials[(int64_t)blockIdx.x * NPART + k] = tot[k];
    }
}

template <int ST>
static hipError_t launch_diag_nodes_s(const DiagNodeLaunch &L, hipStream_t s) {
    using Lay = typename LayoutOf<ST>::L;
    using R = typename LayoutOf<ST>::R;
    using RH = typename LayoutOf<ST>::RH;
    hipLaunchKernelGGL((diag_node_kernel<Lay, R, RH>), dim3(L.nblocks), dim3(MB), 0, s, L.src,
                       (const CavityConst<R> *)L.cav, L.cav_index, L.raw, L.partials, L.tf, L.tm, L.fl_mid);
    return hipGetLastError();
}

hipError_t launch_diag_nodes(const DiagNodeLaunch &L, int nx, int ny, hipStream_t s) {
    if (L.nblocks != diag_node_blocks(nx, ny)) return hipErrorInvalidValue;
    LBM_DISPATCH(L.storage, launch_diag_nodes_s, L, s)
}

// ---------------------------------------------------------------------------
// Initial state.
// ---------------------------------------------------------------------------
template <class Lay, typename R, typename RH>
__global__ __launch_bounds__(MB) void init_kernel(const CavityConst<R> *__restrict__ cav, int ci,
                                                  void *__restrict__ dst, R *__restrict__ sr, int y0, int rows,
                                                  const double *__restrict__ T_pcm,
                                                  const double *__restrict__ T_mf) {
    const CavityConst<R> &c = cav[ci];
    const int nx = c.nx;
    const int64_t nn = (int64_t)nx * rows;
    const int64_t kk = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (kk >= nn) return;
    const double Tf = T_pcm ? T_pcm[kk] : c.T_init;
    const double Tm = T_mf ? T_mf[kk] : c.T_init;
    init_node<Lay, R, RH>(c, dst, sr, (int)(kk % nx), y0 + (int)(kk / nx), Tf, Tm);
}

template <int ST>
static hipError_t launch_init_s(const InitLaunch &L, int nx, hipStream_t s) {
    using Lay = typename LayoutOf<ST>::L;
    using R = typename LayoutOf<ST>::R;
    using RH = typename LayoutOf<ST>::RH;
    hipLaunchKernelGGL((init_kernel<Lay, R, RH>), dim3(row_blocks(nx, L.rows)), dim3(MB), 0, s,
                       (const CavityConst<R> *)L.cav, L.cav_index, L.dst, (R *)L.sr, L.y0, L.rows,
                       L.T_pcm, L.T_mf);
    return hipGetLastError();
}

hipError_t launch_init(const InitLaunch &L, int nx, int ny, hipStream_t s) {
    if (L.y0 < 0 || L.rows < 1 || L.rows > ny - L.y0) return hipErrorInvalidValue;
    LBM_DISPATCH(L.storage, launch_init_s, L, nx, s)
}

// Overwrite one stored element (elem: 8 double, 4 float, 2 binary16,
// 3 bfloat16), for the failure-detection hook.
__global__ void poke_kernel(void *p, int elem, double v) {
    if (elem == 8) *(double *)p = v;
    else if (elem == 4) *(float *)p = (float)v;
    else if (elem == 2) *(uint16_t *)p = E16::enc((float)v);
    else *(uint16_t *)p = EB16::enc((float)v);
}

hipError_t launch_poke(int elem, void *ptr, double value, hipStream_t s) {
    hipLaunchKernelGGL(poke_kernel, dim3(1), dim3(1), 0, s, ptr, elem, value);
    return hipGetLastError();
}

}  // namespace lbm
