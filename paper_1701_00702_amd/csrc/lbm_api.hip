// Host side of the C ABI declared in include/lbmpcm.h: mapping of the
// dimensionless problem to lattice units, device buffers, launch shapes,
// hipGraph replay of the step loop, autotuning, checkpoints and diagnostics.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cstddef>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include <sys/types.h>

#include "../../include/lbmpcm.h"
#include "lbm_internal.h"
#include "lbm_plan.h"

using namespace lbm;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

lbm_status fail(lbm_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(LBM_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),  \
                        __FILE__, __LINE__);                                                 \
    } while (0)

extern "C" const char *lbm_last_error(void) { return g_err; }

// ---------------------------------------------------------------------------
// Device scratch of lbm_diagnostics_noalloc: one fixed array per GPU, held
// until the process ends.  Layout (doubles): per-workgroup partial sums
// [LBM_DIAG_MAX_BLOCKS][NPART], the wall-column temperatures T_f and T_m
// [LBM_NOALLOC_MAX_SIDE][6] each, the middle row's liquid fraction
// [LBM_NOALLOC_MAX_SIDE], the NDIAG results.  In host code the array's name
// is only a stand-in; kernels get the address hipGetSymbolAddress returns
// for the current device (noalloc_scratch).
// ---------------------------------------------------------------------------
#define LBM_NOALLOC_MAX_SIDE 32768
namespace {
constexpr size_t kScrPart = 0;
constexpr size_t kScrTf = kScrPart + (size_t)LBM_DIAG_MAX_BLOCKS * NPART * sizeof(double);
constexpr size_t kScrTm = kScrTf + (size_t)LBM_NOALLOC_MAX_SIDE * 6 * sizeof(double);
constexpr size_t kScrFl = kScrTm + (size_t)LBM_NOALLOC_MAX_SIDE * 6 * sizeof(double);
constexpr size_t kScrOut = kScrFl + (size_t)LBM_NOALLOC_MAX_SIDE * sizeof(double);
constexpr size_t kScrBytes = (kScrOut + 64 * sizeof(double) + 255) & ~(size_t)255;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScrBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// The device address of this GPU's scratch array: looked up once per device
// (with that device current: handle set-up runs on the handle's device).
lbm_status noalloc_scratch(int device, void **out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(LBM_EDEVICE, "device %d beyond the %d devices the scratch table covers", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess || cur != device)
            return fail(LBM_EDEVICE, "scratch of device %d looked up with device %d current", device, cur);
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LBM_EDEVICE, "hipGetSymbolAddress of the diagnostics scratch failed: %s",
                        hipGetErrorString(e));
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return LBM_OK;
}
}  // namespace

namespace {

// Memory plan shared by lbm_workspace_bytes and the create calls.
struct Plan {
    int st = -1;  // storage form (precision and thermal lattice)
    std::vector<Lattice> lat;
    std::vector<int64_t> node0, acc0;
    std::vector<Bands> bands;  // population blocks of each cavity
    int64_t pop_bytes = 0;     // one state buffer
    // nodes: packed index range of the flat per-node arrays (stride each)
    int64_t nodes = 0, stride = 0, slots = 0, max_nodes = 0;
    int max_nx = 0, max_ny = 0;
    // nodes of the staging area that lbm_fields and lbm_set_initial pass
    // whole rows of a cavity through (at least one row of the widest cavity)
    int64_t stage_nodes = 0;
    int max_tiles = 0;
    // tiles of the K-step kernels, K = 2, 3: room for the largest count over
    // the tile shapes (0: not available for this storage)
    int64_t tilesk[4] = {0, 0, 0, 0};
    size_t off_tilesk[4] = {0, 0, 0, 0};
    size_t off_pop[2], off_sr[2], off_acc, off_accs, off_cav, off_tiles, off_fields, off_part, off_tf,
        off_tm, off_fl, off_out, total;
};

// Nodes staged at once: field planes and initial temperatures move between
// host and device in runs of whole rows of at most this many nodes, so the
// staging area stays a small part of the memory however large a cavity is.
constexpr int64_t kStageNodes = (int64_t)1 << 22;

lbm_status make_plan(const lbm_params *p, int n, lbm_precision prec, Plan &pl) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (n < 1) return fail(LBM_EINVAL, "need at least one cavity");
    if (storage_of(prec) < 0) return fail(LBM_EINVAL, "unknown precision %d", (int)prec);
    const int qt0 = p[0].thermal_lattice == 5 ? 5 : 9;
    for (int c = 1; c < n; ++c)
        if ((p[c].thermal_lattice == 5 ? 5 : 9) != qt0)
            return fail(LBM_EINVAL, "cavity %d: every cavity of a batch needs the same thermal lattice", c);
    pl.lat.resize(n);
    int64_t tiles = 0;
    for (int c = 0; c < n; ++c) {
        lbm_status s = map_params(p[c], prec, pl.lat[c]);
        if (s != LBM_OK) {
            char buf[512];
            snprintf(buf, sizeof(buf), "cavity %d: %s", c, g_err);
            return fail(s, "%s", buf);
        }
        pl.node0.push_back(pl.nodes);
        pl.acc0.push_back(pl.slots);
        const int64_t nn = (int64_t)p[c].nx * p[c].ny;
        // each cavity starts on a 64-node boundary, so aligned tiles store
        // whole cache lines
        pl.nodes += (nn + 63) & ~(int64_t)63;
        pl.slots += 2 * ((int64_t)p[c].nx + p[c].ny);
        pl.max_nodes = std::max(pl.max_nodes, nn);
        pl.max_nx = std::max(pl.max_nx, p[c].nx);
        pl.max_ny = std::max(pl.max_ny, p[c].ny);
        // interior rows and the wall ring, in tiles of at least 64 nodes
        const int64_t pitch = (p[c].nx + 63) & ~63;
        tiles += (pitch * (p[c].ny - 2) + 63) / 64 + 1 + 2 * (((int64_t)p[c].nx + 63) / 64);
    }
    if (pl.nodes >= ((int64_t)1 << 31) - 1024) return fail(LBM_EINVAL, "more than 2^31 nodes in total");
    if (tiles >= ((int64_t)1 << 31)) return fail(LBM_EINVAL, "too many tiles");
    pl.max_tiles = (int)tiles;
    pl.st = storage_of(prec, qt0);
    const int st = pl.st;
    pl.stride = (pl.nodes + 127) & ~(int64_t)127;
    for (int c = 0; c < n; ++c) {
        const Bands b = bands_of(p[c].nx, p[c].ny, bytes_per_node(st), pl.pop_bytes, p[c].band_rows);
        // the step kernels' 32-bit offsets within two consecutive blocks
        if (b.nodes * (bytes_per_node(st) + 8) >= ((int64_t)1 << 31))
            return fail(LBM_EINVAL, "cavity %d: rows of %d nodes are too long", c, p[c].nx);
        pl.bands.push_back(b);
        pl.pop_bytes += b.bytes * b.count;
    }
    size_t off = 0;
    for (int b = 0; b < 2; ++b) {
        pl.off_pop[b] = off;
        off = align256(off + (size_t)pl.pop_bytes);
    }
    for (int b = 0; b < 2; ++b) {
        pl.off_sr[b] = off;
        off = align256(off + (size_t)pl.stride * real_size(st));
    }
    pl.off_acc = off;
    off = align256(off + (size_t)pl.slots * 2 * sizeof(double));
    pl.off_accs = off;
    off = align256(off + (size_t)pl.slots * 2 * sizeof(double));
    pl.off_cav = off;
    off = align256(off + (size_t)n * std::max(sizeof(CavityConst<double>), sizeof(CavityConst<float>)));
    pl.off_tiles = off;
    off = align256(off + (size_t)pl.max_tiles * sizeof(Tile));
    for (int k = 2; k <= 3; ++k) {
        if (!stepk_supported(st, k)) continue;
        for (int shape = 0; shape < LBM_TILE_SHAPES; ++shape) {
            int tw, th;
            stepk_tile(st, k, shape, &tw, &th);
            int64_t count = 0;
            for (int c = 0; c < n; ++c) count += count_tiles2(p[c].nx, p[c].ny, tw, th);
            pl.tilesk[k] = std::max(pl.tilesk[k], count);
        }
        if (pl.tilesk[k] >= ((int64_t)1 << 31)) return fail(LBM_EINVAL, "too many tiles");
        pl.off_tilesk[k] = off;
        off = align256(off + (size_t)pl.tilesk[k] * sizeof(Tile2));
    }
    pl.stage_nodes = std::max<int64_t>(std::min(pl.max_nodes, kStageNodes), pl.max_nx);
    pl.off_fields = off;
    off = align256(off + (size_t)6 * pl.stage_nodes * sizeof(double));
    pl.off_part = off;
    off = align256(off + (size_t)LBM_DIAG_MAX_BLOCKS * NPART * sizeof(double));
    pl.off_tf = off;
    off = align256(off + (size_t)pl.max_ny * 6 * sizeof(double));
    pl.off_tm = off;
    off = align256(off + (size_t)pl.max_ny * 6 * sizeof(double));
    pl.off_fl = off;
    off = align256(off + (size_t)pl.max_nx * sizeof(double));
    pl.off_out = off;
    off = align256(off + 64 * sizeof(double));
    pl.total = off;
    return LBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
struct lbm_handle {
    Plan pl;
    lbm_precision prec;
    int st;
    int n;
    std::vector<lbm_params> params;
    char *ws = nullptr;
    bool owns_ws = false;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    hipStream_t cap = nullptr;
    int device = 0;
    int n_cu = 256;
    int cur = 0;
    int64_t step = 0;
    std::vector<double> E0, M0;
    lbm_launch_config lc{512, 1, 1, 0, 1, 0, 0, 0};
    int ntk[4] = {0, 0, 0, 0};     // tiles in the K-step tables (K = 2, 3)
    int shapek[4] = {0, 0, 0, 0};  // tile shape the K-step tables were built for
    std::vector<Tile> tiles;             // host copy, sorted by cavity: interior, then ring
    std::vector<int> cav_tile0, cav_ntiles;
    int graph_chunk = 32;  // launches per captured graph
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipGraph_t gsrc[2] = {nullptr, nullptr};
    hipGraphExec_t graphk[4][2] = {};  // K-step launches, K = 2, 3
    hipGraph_t gsrck[4][2] = {};

    void *pop(int b) { return ws + pl.off_pop[b]; }
    void *sr(int b) { return ws + pl.off_sr[b]; }
    double *acc() { return (double *)(ws + pl.off_acc); }
    double *acc_scratch() { return (double *)(ws + pl.off_accs); }
    void *cav() { return ws + pl.off_cav; }
    Tile *dtiles() { return (Tile *)(ws + pl.off_tiles); }
    Tile2 *dtilesk(int k) { return (Tile2 *)(ws + pl.off_tilesk[k]); }
    double *fields() { return (double *)(ws + pl.off_fields); }
    double *dout() { return (double *)(ws + pl.off_out); }
    // rows of cavity c that fit the staging area at once
    int stage_rows(int c) const {
        const lbm_params &p = params[c];
        return (int)std::min<int64_t>(p.ny, std::max<int64_t>(1, pl.stage_nodes / p.nx));
    }
};

namespace {

void drop_graphs(lbm_handle *h) {
    for (int b = 0; b < 2; ++b) {
        if (h->graph[b]) (void)hipGraphExecDestroy(h->graph[b]);
        if (h->gsrc[b]) (void)hipGraphDestroy(h->gsrc[b]);
        h->graph[b] = nullptr;
        h->gsrc[b] = nullptr;
        for (int k = 2; k <= 3; ++k) {
            if (h->graphk[k][b]) (void)hipGraphExecDestroy(h->graphk[k][b]);
            if (h->gsrck[k][b]) (void)hipGraphDestroy(h->gsrck[k][b]);
            h->graphk[k][b] = nullptr;
            h->gsrck[k][b] = nullptr;
        }
    }
}

// Tile table of the K-step kernel in tile shape `shape`.
lbm_status build_tilesk(lbm_handle *h, int k, int shape) {
    if (!h->pl.tilesk[k]) return LBM_OK;
    int tw, th;
    stepk_tile(h->st, k, shape, &tw, &th);
    if (!tw) return fail(LBM_EINVAL, "no tile shape %d for %d steps per launch", shape, k);
    std::vector<Tile2> t;
    for (int c = 0; c < h->n; ++c) cavity_tiles2(c, h->params[c].nx, h->params[c].ny, tw, th, t);
    if ((int64_t)t.size() > h->pl.tilesk[k]) return fail(LBM_EINVAL, "K-step tile table overflow");
    HIP_TRY(hipMemcpyAsync(h->dtilesk(k), t.data(), t.size() * sizeof(Tile2), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->ntk[k] = (int)t.size();
    h->shapek[k] = shape;
    return LBM_OK;
}

// The K-step tables a launch shape needs: its own K in its tile shape, and
// with three steps per launch the two-step table (default shape) for a
// remainder of two steps.
lbm_status tables_for(lbm_handle *h, const lbm_launch_config &lc) {
    for (int k = 2; k <= 3; ++k) {
        const int shape = lc.steps_per_launch == k ? lc.tile_shape : 0;
        if (h->pl.tilesk[k] && (h->ntk[k] == 0 || h->shapek[k] != shape)) {
            lbm_status s = build_tilesk(h, k, shape);
            if (s != LBM_OK) return s;
        }
    }
    return LBM_OK;
}

lbm_status build_tiles(lbm_handle *h, const lbm_launch_config &lc) {
    const int tw = lc.block * lc.nodes_per_thread;
    h->tiles.clear();
    h->cav_tile0.assign(h->n, 0);
    h->cav_ntiles.assign(h->n, 0);
    for (int c = 0; c < h->n; ++c) {
        h->cav_tile0[c] = (int)h->tiles.size();
        const int nx = h->params[c].nx, ny = h->params[c].ny;
        const int pitch = h->pl.bands[c].pitch;
        // interior tiles run over the pitched index k = y * pitch + x of
        // rows 1..ny-2 (rows start on 64-node boundaries, so every wavefront
        // stores whole cache lines; lanes on the padding idle)
        for (int k0 = pitch; k0 < pitch * (ny - 1); k0 += tw)
            h->tiles.push_back(Tile{c, TILE_INTERIOR, k0, std::min(pitch * (ny - 1), k0 + tw)});
        // wall tiles hold nodes of one row (the bottom or the top)
        for (int row = 0; row < 2; ++row)
            for (int r0 = row * nx; r0 < (row + 1) * nx; r0 += tw)
                h->tiles.push_back(Tile{c, TILE_WALL, r0, std::min((row + 1) * nx, r0 + tw)});
        h->cav_ntiles[c] = (int)h->tiles.size() - h->cav_tile0[c];
    }
    if ((int)h->tiles.size() > h->pl.max_tiles) return fail(LBM_EINVAL, "tile table overflow");
    HIP_TRY(hipMemcpyAsync(h->dtiles(), h->tiles.data(), h->tiles.size() * sizeof(Tile),
                           hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// whether the plan has the tiles of K steps per launch
bool has_k(const Plan &pl, int k) { return k == 1 || ((k == 2 || k == 3) && pl.tilesk[k] > 0); }

bool valid_launch(const lbm_launch_config &lc, const Plan &pl) {
    const bool b = lc.block == 64 || lc.block == 128 || lc.block == 256 || lc.block == 512;
    const bool n = lc.nodes_per_thread == 1 || lc.nodes_per_thread == 2 || lc.nodes_per_thread == 4;
    const bool t = has_k(pl, lc.steps_per_launch);
    // alternative tile shapes: multi-step launches without a persistent grid
    const bool sh = lc.tile_shape == 0 ||
                    (lc.tile_shape > 0 && lc.tile_shape < LBM_TILE_SHAPES && lc.steps_per_launch > 1 &&
                     lc.persistent == 0);
    return b && n && t && sh && (lc.xcd_remap == 0 || lc.xcd_remap == 1) && lc.persistent >= 0 &&
           lc.persistent <= 64;
}

// The launch shape as reported: the tile dimensions of the multi-step
// kernel filled in.
lbm_launch_config reported(const lbm_handle *h, lbm_launch_config lc) {
    lc.tile_w = lc.tile_h = 0;
    if (lc.steps_per_launch > 1) stepk_tile(h->st, lc.steps_per_launch, lc.tile_shape, &lc.tile_w, &lc.tile_h);
    return lc;
}

Step2Launch stepk_args(lbm_handle *h, int k, int src_buf, double *acc, const lbm_launch_config &lc) {
    Step2Launch L;
    L.storage = h->st;
    L.steps = k;
    L.shape = h->shapek[k];
    const int nt = h->ntk[k];
    L.grid = lc.persistent > 0 ? std::min(nt, h->n_cu * lc.persistent) : nt;
    L.xcd_remap = lc.xcd_remap;
    L.src = h->pop(src_buf);
    L.dst = h->pop(1 - src_buf);
    L.sr_src = h->sr(src_buf);
    L.sr_dst = h->sr(1 - src_buf);
    L.acc = acc;
    L.cav = h->cav();
    L.tiles = h->dtilesk(k);
    L.ntiles = nt;
    return L;
}

StepLaunch step_args(lbm_handle *h, int pull, int src_buf, double *acc, int tile0, int ntiles,
                     const lbm_launch_config &lc) {
    StepLaunch L;
    L.storage = h->st;
    L.block = lc.block;
    L.npt = lc.nodes_per_thread;
    L.xcd_remap = lc.xcd_remap;
    L.grid = lc.persistent > 0 ? std::min(ntiles, h->n_cu * lc.persistent) : ntiles;
    L.pull = pull;
    L.src = h->pop(src_buf);
    L.dst = h->pop(1 - src_buf);
    L.sr_src = h->sr(src_buf);
    L.sr_dst = h->sr(1 - src_buf);
    L.acc = acc;
    L.cav = h->cav();
    L.tiles = h->dtiles() + tile0;
    L.ntiles = ntiles;
    return L;
}

lbm_status launch_one(lbm_handle *h, hipStream_t s, int pull, int src_buf) {
    StepLaunch L = step_args(h, pull, src_buf, h->acc(), 0, (int)h->tiles.size(), h->lc);
    HIP_TRY(launch_step(L, s));
    return LBM_OK;
}

// Graph of graph_chunk launches of K steps each (K = 1: the one-step kernel).
lbm_status build_graph(lbm_handle *h, int parity, int kk) {
    if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    int b = parity;
    for (int k = 0; k < h->graph_chunk; ++k) {
        hipError_t e;
        if (kk > 1) {
            Step2Launch L = stepk_args(h, kk, b, h->acc(), h->lc);
            e = launch_stepk(L, h->cap);
        } else {
            StepLaunch L = step_args(h, 1, b, h->acc(), 0, (int)h->tiles.size(), h->lc);
            e = launch_step(L, h->cap);
        }
        if (e != hipSuccess) {
            hipGraph_t g;
            (void)hipStreamEndCapture(h->cap, &g);
            if (g) (void)hipGraphDestroy(g);
            return fail(LBM_EDEVICE, "kernel launch during capture failed: %s", hipGetErrorString(e));
        }
        b ^= 1;
    }
    hipGraph_t *src = kk > 1 ? &h->gsrck[kk][parity] : &h->gsrc[parity];
    hipGraphExec_t *ex = kk > 1 ? &h->graphk[kk][parity] : &h->graph[parity];
    HIP_TRY(hipStreamEndCapture(h->cap, src));
    HIP_TRY(hipGraphInstantiate(ex, *src, nullptr, nullptr, 0));
    return LBM_OK;
}

// Capture both parities' graphs of the current launch mode now (creation and
// every change of launch shape), so that no lbm_step spends host time on
// capture and instantiation while the device waits.
lbm_status prepare_graphs(lbm_handle *h) {
    const int kk = h->lc.steps_per_launch;
    for (int parity = 0; parity < 2; ++parity) {
        if (kk > 1 ? h->graphk[kk][parity] : h->graph[parity]) continue;
        lbm_status s = build_graph(h, parity, kk);
        if (s != LBM_OK) return s;
    }
    return LBM_OK;
}

// Arguments of the final diagnostics pass of cavity c (everything but the
// wall-column and middle-row pointers).
DiagLaunch diag_args(lbm_handle *h, int c, const double *partials, int nblocks, double *out) {
    const lbm_params &p = h->params[c];
    const Lattice &l = h->pl.lat[c];
    DiagLaunch D;
    std::memset(&D, 0, sizeof(D));
    D.nx = p.nx;
    D.ny = p.ny;
    D.periodic = p.bc_x;
    D.acc0 = h->pl.acc0[c];
    D.partials = partials;
    D.nblocks = nblocks;
    D.acc = h->acc();
    D.out = out;
    D.L = l.L;
    D.kf = l.phi * l.k_f;
    D.km = (1.0 - l.phi) * l.k_m;
    D.ke = D.kf + D.km;
    D.dT = l.T_hot - l.T_cold;
    return D;
}

// The diagnostics kernels of cavity c, their scratch at the given device
// addresses: per-workgroup partial sums, the temperatures of the columns
// next to the vertical walls, the middle row's liquid fraction, and the
// NDIAG results in out.
lbm_status launch_diagnostics(lbm_handle *h, int c, char *part, char *tf, char *tm, char *fl, char *out) {
    const lbm_params &p = h->params[c];
    DiagNodeLaunch M;
    M.storage = h->st;
    M.raw = h->step == 0 ? 1 : 0;
    M.cav_index = c;
    M.src = h->pop(h->cur);
    M.cav = h->cav();
    M.partials = (double *)part;
    M.nblocks = diag_node_blocks(p.nx, p.ny);
    M.tf = (double *)tf;
    M.tm = (double *)tm;
    M.fl_mid = (double *)fl;
    HIP_TRY(launch_diag_nodes(M, p.nx, p.ny, h->stream));
    DiagLaunch D = diag_args(h, c, M.partials, M.nblocks, (double *)out);
    D.tf = M.tf;
    D.tm = M.tm;
    D.fl_mid = M.fl_mid;
    HIP_TRY(launch_diag(D, p.nx, p.ny, h->stream));
    return LBM_OK;
}

// Diagnostics of cavity c with the workspace as scratch, copied to out.
lbm_status read_diag(lbm_handle *h, int c, double out[NDIAG]) {
    char *w = h->ws;
    lbm_status s = launch_diagnostics(h, c, w + h->pl.off_part, w + h->pl.off_tf, w + h->pl.off_tm,
                                      w + h->pl.off_fl, w + h->pl.off_out);
    if (s != LBM_OK) return s;
    HIP_TRY(hipMemcpyAsync(out, h->dout(), NDIAG * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

lbm_status init_cavity(lbm_handle *h, int c, const double *T_pcm, const double *T_mf) {
    const lbm_params &p = h->params[c];
    const int chunk = h->stage_rows(c);
    double *dT = h->fields();  // staging for the temperature arrays
    // runs of whole rows through the staging area; stream order keeps a
    // run's copies behind the previous run's kernel
    for (int y0 = 0; y0 < p.ny; y0 += chunk) {
        const int rows = std::min(chunk, p.ny - y0);
        const int64_t nn = (int64_t)p.nx * rows, o = (int64_t)p.nx * y0;
        if (T_pcm)
            HIP_TRY(hipMemcpyAsync(dT, T_pcm + o, nn * sizeof(double), hipMemcpyHostToDevice, h->stream));
        if (T_mf)
            HIP_TRY(hipMemcpyAsync(dT + nn, T_mf + o, nn * sizeof(double), hipMemcpyHostToDevice, h->stream));
        InitLaunch I;
        I.storage = h->st;
        I.cav_index = c;
        I.cav = h->cav();
        I.dst = h->pop(h->cur);
        I.sr = h->sr(h->cur);
        I.y0 = y0;
        I.rows = rows;
        I.T_pcm = T_pcm ? dT : nullptr;
        I.T_mf = T_mf ? dT + nn : nullptr;
        HIP_TRY(launch_init(I, p.nx, p.ny, h->stream));
    }
    const int64_t a0 = h->pl.acc0[c], ns = 2 * ((int64_t)p.nx + p.ny);
    HIP_TRY(hipMemsetAsync(h->acc() + 2 * a0, 0, ns * 2 * sizeof(double), h->stream));
    double d[NDIAG];
    lbm_status s = read_diag(h, c, d);
    if (s != LBM_OK) return s;
    h->E0[c] = d[D_E];
    h->M0[c] = d[D_M];
    return LBM_OK;
}

lbm_status setup(lbm_handle *h) {
    HIP_TRY(hipGetDevice(&h->device));
    {
        void *scr = nullptr;
        lbm_status s0 = noalloc_scratch(h->device, &scr);
        if (s0 != LBM_OK) return s0;
    }
    int ncu = 0;
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
    h->n_cu = ncu > 0 ? ncu : 256;
    HIP_TRY(hipMemsetAsync(h->ws, 0, h->pl.total, h->stream));
    // cavity table in the kernels' arithmetic type (FP64 forms: double)
    if (real_size(h->st) == 8) {
        std::vector<CavityConst<double>> t;
        for (int c = 0; c < h->n; ++c)
            t.push_back(make_const<double>(h->pl.lat[c], h->pl.node0[c], h->pl.acc0[c], h->pl.bands[c]));
        HIP_TRY(hipMemcpyAsync(h->cav(), t.data(), t.size() * sizeof(t[0]), hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    } else {
        std::vector<CavityConst<float>> t;
        for (int c = 0; c < h->n; ++c)
            t.push_back(make_const<float>(h->pl.lat[c], h->pl.node0[c], h->pl.acc0[c], h->pl.bands[c]));
        HIP_TRY(hipMemcpyAsync(h->cav(), t.data(), t.size() * sizeof(t[0]), hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    // By default the most steps per launch the form has (measured faster
    // for every cavity size and batch, the rows being padded to 64 nodes).
    h->lc.steps_per_launch = h->pl.tilesk[3] > 0 ? 3 : (h->pl.tilesk[2] > 0 ? 2 : 1);
    lbm_status s = build_tiles(h, h->lc);
    if (s != LBM_OK) return s;
    s = tables_for(h, h->lc);
    if (s != LBM_OK) return s;
    h->E0.assign(h->n, 0.0);
    h->M0.assign(h->n, 0.0);
    for (int c = 0; c < h->n; ++c) {
        s = init_cavity(h, c, nullptr, nullptr);
        if (s != LBM_OK) return s;
    }
    return prepare_graphs(h);
}

lbm_status create_common(const lbm_params *p, int n, lbm_precision prec, void *ws, uint64_t ws_bytes,
                         void *stream, bool ext, lbm_handle **out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    lbm_handle *h = new lbm_handle();
    lbm_status s = make_plan(p, n, prec, h->pl);
    if (s != LBM_OK) {
        delete h;
        return s;
    }
    h->prec = prec;
    h->st = h->pl.st;
    h->n = n;
    for (int c = 0; c < n; ++c) h->params.push_back(normalized(p[c]));
    h->stream = (hipStream_t)stream;
    if (ext) {
        if (!ws) {
            delete h;
            return fail(LBM_EINVAL, "workspace is NULL");
        }
        if (ws_bytes < h->pl.total) {
            delete h;
            return fail(LBM_EINVAL, "workspace of %llu bytes is smaller than the %llu needed",
                        (unsigned long long)ws_bytes, (unsigned long long)h->pl.total);
        }
        if (((uintptr_t)ws) & 255) {
            delete h;
            return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
        }
        h->ws = (char *)ws;
    } else {
        hipError_t e = hipMalloc((void **)&h->ws, h->pl.total);
        if (e != hipSuccess) {
            delete h;
            return fail(LBM_ENOMEM, "hipMalloc of %llu bytes failed: %s", (unsigned long long)h->pl.total,
                        hipGetErrorString(e));
        }
        h->owns_ws = true;
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            (void)hipFree(h->ws);
            delete h;
            return fail(LBM_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
        }
        h->owns_stream = true;
    }
    s = setup(h);
    if (s != LBM_OK) {
        std::string msg = g_err;
        lbm_destroy(h);
        return fail(s, "%s", msg.c_str());
    }
    *out = h;
    return LBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" lbm_status lbm_workspace_bytes(const lbm_params *p, int32_t n, lbm_precision prec,
                                          uint64_t *bytes) {
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    Plan pl;
    lbm_status s = make_plan(p, n, prec, pl);
    if (s != LBM_OK) return s;
    *bytes = pl.total;
    return LBM_OK;
}

extern "C" lbm_status lbm_create(const lbm_params *p, lbm_precision prec, lbm_handle **out) {
    return create_common(p, 1, prec, nullptr, 0, nullptr, false, out);
}

extern "C" lbm_status lbm_create_batch(const lbm_params *p, int32_t n, lbm_precision prec,
                                       lbm_handle **out) {
    return create_common(p, n, prec, nullptr, 0, nullptr, false, out);
}

extern "C" lbm_status lbm_create_ext(const lbm_params *p, int32_t n, lbm_precision prec, void *ws,
                                     uint64_t ws_bytes, void *stream, lbm_handle **out) {
    return create_common(p, n, prec, ws, ws_bytes, stream, true, out);
}

extern "C" lbm_status lbm_destroy(lbm_handle *h) {
    if (!h) return LBM_OK;
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->owns_stream && h->stream) (void)hipStreamDestroy(h->stream);
    if (h->owns_ws && h->ws) (void)hipFree(h->ws);
    delete h;
    return LBM_OK;
}

extern "C" lbm_status lbm_set_stream(lbm_handle *h, void *stream) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (h->owns_stream && h->stream) HIP_TRY(hipStreamDestroy(h->stream));
    h->owns_stream = false;  // the caller's stream is never destroyed here
    h->stream = (hipStream_t)stream;
    return LBM_OK;
}

extern "C" lbm_status lbm_set_initial(lbm_handle *h, int32_t c, const double *T_pcm, const double *T_mf) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (c < 0 || c >= h->n) return fail(LBM_EINVAL, "cavity %d out of range", c);
    if (h->step != 0) return fail(LBM_ESTATE, "initial state can only be set before the first step");
    return init_cavity(h, c, T_pcm, T_mf);
}

extern "C" lbm_status lbm_step(lbm_handle *h, int64_t n) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (n < 0) return fail(LBM_EINVAL, "negative step count");
    if (n == 0) return LBM_OK;
    if (h->step == 0) {
        lbm_status s = launch_one(h, h->stream, 0, h->cur);
        if (s != LBM_OK) return s;
        h->cur ^= 1;
        h->step += 1;
        n -= 1;
    }
    const int kk = h->lc.steps_per_launch;
    if (kk > 1) {
        // runs of kk steps, one launch each (a launch swaps the buffers once)
        while (n >= (int64_t)kk * h->graph_chunk && h->graph_chunk > 0) {
            if (!h->graphk[kk][h->cur]) {
                lbm_status s = build_graph(h, h->cur, kk);
                if (s != LBM_OK) return s;
            }
            HIP_TRY(hipGraphLaunch(h->graphk[kk][h->cur], h->stream));
            if (h->graph_chunk & 1) h->cur ^= 1;  // each captured launch swaps the buffers
            h->step += (int64_t)kk * h->graph_chunk;
            n -= (int64_t)kk * h->graph_chunk;
        }
        for (; n >= kk; n -= kk) {
            Step2Launch L = stepk_args(h, kk, h->cur, h->acc(), h->lc);
            HIP_TRY(launch_stepk(L, h->stream));
            h->cur ^= 1;
            h->step += kk;
        }
        // two steps left of three-step runs: one two-step launch
        if (n == 2 && kk == 3 && h->pl.tilesk[2] > 0) {
            Step2Launch L = stepk_args(h, 2, h->cur, h->acc(), h->lc);
            HIP_TRY(launch_stepk(L, h->stream));
            h->cur ^= 1;
            h->step += 2;
            n -= 2;
        }
    }
    while (n >= h->graph_chunk && h->graph_chunk > 0) {
        if (!h->graph[h->cur]) {
            lbm_status s = build_graph(h, h->cur, 1);
            if (s != LBM_OK) return s;
        }
        HIP_TRY(hipGraphLaunch(h->graph[h->cur], h->stream));
        if (h->graph_chunk & 1) h->cur ^= 1;
        h->step += h->graph_chunk;
        n -= h->graph_chunk;
    }
    for (; n > 0; --n) {
        lbm_status s = launch_one(h, h->stream, 1, h->cur);
        if (s != LBM_OK) return s;
        h->cur ^= 1;
        h->step += 1;
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_step_per_cavity(lbm_handle *h, int64_t n) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (n < 0) return fail(LBM_EINVAL, "negative step count");
    for (int64_t k = 0; k < n; ++k) {
        const int pull = h->step == 0 ? 0 : 1;
        for (int c = 0; c < h->n; ++c) {
            StepLaunch L = step_args(h, pull, h->cur, h->acc(), h->cav_tile0[c], h->cav_ntiles[c], h->lc);
            HIP_TRY(launch_step(L, h->stream));
        }
        h->cur ^= 1;
        h->step += 1;
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_synchronize(lbm_handle *h) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

extern "C" int64_t lbm_step_count(const lbm_handle *h) { return h ? h->step : -1; }

extern "C" lbm_status lbm_fields_rows(lbm_handle *h, int32_t c, int32_t y0, int32_t rows, double *ux,
                                      double *uy, double *T_pcm, double *T_mf, double *f_l, double *rho) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (c < 0 || c >= h->n) return fail(LBM_EINVAL, "cavity %d out of range", c);
    const lbm_params &p = h->params[c];
    if (y0 < 0 || rows < 1 || rows > p.ny - y0)
        return fail(LBM_EINVAL, "rows [%d, %d + %d) outside the cavity's %d rows", y0, y0, rows, p.ny);
    const int chunk = h->stage_rows(c);
    double *outs[6] = {ux, uy, T_pcm, T_mf, f_l, rho};
    for (int r0 = 0; r0 < rows; r0 += chunk) {
        const int nr = std::min(chunk, rows - r0);
        MacroLaunch M;
        M.storage = h->st;
        M.raw = h->step == 0 ? 1 : 0;
        M.cav_index = c;
        M.src = h->pop(h->cur);
        M.cav = h->cav();
        M.y0 = y0 + r0;
        M.rows = nr;
        M.fields = h->fields();
        HIP_TRY(launch_macro(M, p.nx, p.ny, h->stream));
        const int64_t nn = (int64_t)p.nx * nr;
        for (int k = 0; k < 6; ++k)
            if (outs[k])
                HIP_TRY(hipMemcpyAsync(outs[k] + (int64_t)p.nx * r0, h->fields() + k * nn, nn * sizeof(double),
                                       hipMemcpyDeviceToHost, h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

extern "C" lbm_status lbm_fields(lbm_handle *h, int32_t c, double *ux, double *uy, double *T_pcm,
                                 double *T_mf, double *f_l, double *rho) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (c < 0 || c >= h->n) return fail(LBM_EINVAL, "cavity %d out of range", c);
    return lbm_fields_rows(h, c, 0, h->params[c].ny, ux, uy, T_pcm, T_mf, f_l, rho);
}

namespace {
// lbm_diag of cavity c from the device results d (NDIAG doubles).
lbm_status diag_from(lbm_handle *h, int c, const double d[NDIAG], lbm_diag *out) {
    const Lattice &l = h->pl.lat[c];
    std::memset(out, 0, sizeof(*out));
    out->step = (double)h->step;
    out->Fo = (double)h->step * (l.k_f / (l.rho_l * l.c_pl)) / (l.L * l.L);
    out->liquid_fraction = d[D_FL];
    out->Nu_hot = d[D_NUH];
    out->Nu_hot_pcm = d[D_NUHP];
    out->Nu_cold = d[D_NUC];
    out->E_int = d[D_E];
    out->E_int0 = h->E0[c];
    out->M_int = d[D_M];
    out->M_int0 = h->M0[c];
    double sE = 0, sM = 0;
    for (int w = 0; w < 4; ++w) {
        out->flux_E[w] = d[D_FLUXE + w];
        out->flux_M[w] = d[D_FLUXM + w];
        sE += d[D_FLUXE + w];
        sM += d[D_FLUXM + w];
    }
    out->energy_residual = out->E_int - out->E_int0 - sE;
    out->mass_residual = out->M_int - out->M_int0 - sM;
    out->x_front_mid = d[D_FRONT];
    out->max_dT_LTNE = d[D_DT];
    out->u_max = d[D_U];
    out->nonfinite = d[D_NF];
    if (d[D_NF] > 0) return fail(LBM_ENONFINITE, "cavity %d holds %g nodes with non-finite populations", c, d[D_NF]);
    return LBM_OK;
}
}  // namespace

extern "C" lbm_status lbm_diagnostics(lbm_handle *h, int32_t c, lbm_diag *out) {
    if (!h || !out) return fail(LBM_EINVAL, "NULL argument");
    if (c < 0 || c >= h->n) return fail(LBM_EINVAL, "cavity %d out of range", c);
    double d[NDIAG];
    lbm_status s = read_diag(h, c, d);
    if (s != LBM_OK) return s;
    return diag_from(h, c, d, out);
}

extern "C" lbm_status lbm_diagnostics_noalloc(lbm_handle *h, int32_t c, lbm_diag *out) {
    if (!h || !out) return fail(LBM_EINVAL, "NULL argument");
    if (c < 0 || c >= h->n) return fail(LBM_EINVAL, "cavity %d out of range", c);
    const lbm_params &p = h->params[c];
    if (p.nx > LBM_NOALLOC_MAX_SIDE || p.ny > LBM_NOALLOC_MAX_SIDE)
        return fail(LBM_EINVAL, "cavity %d is %dx%d: lbm_diagnostics_noalloc takes sides of at most %d nodes "
                    "(its fixed scratch); use lbm_diagnostics", c, p.nx, p.ny, LBM_NOALLOC_MAX_SIDE);
    void *scr = nullptr;
    lbm_status s = noalloc_scratch(h->device, &scr);
    if (s != LBM_OK) return s;
    char *base = (char *)scr;
    s = launch_diagnostics(h, c, base + kScrPart, base + kScrTf, base + kScrTm, base + kScrFl, base + kScrOut);
    if (s != LBM_OK) return s;
    double d[NDIAG];
    HIP_TRY(hipMemcpyAsync(d, base + kScrOut, NDIAG * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return diag_from(h, c, d, out);
}

namespace {
void fill_lattice(const Lattice &l, lbm_lattice *out) {
    std::memset(out, 0, sizeof(*out));
    out->L = l.L;
    out->k_f = l.k_f;
    out->k_m = l.k_m;
    out->nu_f = l.nu_f;
    out->nu_e = l.nu_e;
    out->K = l.K;
    out->F_phi = l.F_phi;
    out->gbeta = l.gbeta;
    out->h_v = l.h_v;
    out->L_a = l.L_a;
    out->d_p = l.d_p;
    out->z = l.z;
    out->tau_v = 1.0 / l.s[7];
    out->tau_g = 1.0 / l.zeta_a;
    out->tau_h = 1.0 / l.eta_a;
    for (int k = 0; k < 9; ++k) {
        out->s[k] = l.s[k];
        out->zeta[k] = l.zeta[k];
        out->eta[k] = l.eta[k];
    }
    out->H_fs = l.H_fs;
    out->H_fl = l.H_fl;
    out->T_ref = l.T_ref;
    out->H_ref = l.H_ref;
    for (int f = 0; f < 3; ++f) out->scale_exp[f] = l.scale_exp[f];
    out->q_thermal = l.qt;
    out->varpi = l.varpi;
    for (int w = 0; w < 4; ++w) {
        out->wall_type[w] = l.wall_type[w];
        out->wall_T[w] = l.wall_T[w];
    }
    out->solid_treatment = l.solid;
}
}  // namespace

extern "C" lbm_status lbm_get_lattice(const lbm_handle *h, int32_t c, lbm_lattice *out) {
    if (!h || !out) return fail(LBM_EINVAL, "NULL argument");
    if (c < 0 || c >= h->n) return fail(LBM_EINVAL, "cavity %d out of range", c);
    fill_lattice(h->pl.lat[c], out);
    return LBM_OK;
}

extern "C" lbm_status lbm_lattice_of(const lbm_params *p, lbm_precision prec, lbm_lattice *out) {
    if (!p || !out) return fail(LBM_EINVAL, "NULL argument");
    if (storage_of(prec) < 0) return fail(LBM_EINVAL, "unknown precision %d", (int)prec);
    Lattice l;
    lbm_status s = map_params(*p, prec, l);
    if (s != LBM_OK) return s;
    fill_lattice(l, out);
    return LBM_OK;
}

extern "C" lbm_status lbm_get_launch(const lbm_handle *h, lbm_launch_config *out) {
    if (!h || !out) return fail(LBM_EINVAL, "NULL argument");
    *out = reported(h, h->lc);
    return LBM_OK;
}

extern "C" lbm_status lbm_set_launch(lbm_handle *h, const lbm_launch_config *cfg) {
    if (!h || !cfg) return fail(LBM_EINVAL, "NULL argument");
    if (!valid_launch(*cfg, h->pl))
        return fail(LBM_EINVAL,
                    "unsupported launch shape block=%d npt=%d xcd=%d persistent=%d steps=%d tile_shape=%d",
                    cfg->block, cfg->nodes_per_thread, cfg->xcd_remap, cfg->persistent, cfg->steps_per_launch,
                    cfg->tile_shape);
    HIP_TRY(hipStreamSynchronize(h->stream));
    lbm_status s = build_tiles(h, *cfg);
    if (s != LBM_OK) return s;
    s = tables_for(h, *cfg);
    if (s != LBM_OK) return s;
    h->lc = reported(h, *cfg);
    drop_graphs(h);
    return prepare_graphs(h);
}

namespace {
std::string tune_key(lbm_handle *h) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    char buf[256];
    snprintf(buf, sizeof(buf), "%s:st%d:n%d:nodes%lld:nx%d:ny%d", arch.c_str(), h->st, h->n,
             (long long)h->pl.nodes, h->params[0].nx, h->params[0].ny);
    return buf;
}
}  // namespace

extern "C" lbm_status lbm_autotune(lbm_handle *h, int32_t steps, const char *cache_path,
                                   lbm_launch_config *chosen) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (steps < 1) return fail(LBM_EINVAL, "steps_per_trial must be >= 1");
    const std::string key = tune_key(h);
    if (cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char k[256];
            lbm_launch_config lc;
            std::memset(&lc, 0, sizeof(lc));
            while (fscanf(f, "%255s %d %d %d %d %d %d", k, &lc.block, &lc.nodes_per_thread, &lc.xcd_remap,
                          &lc.persistent, &lc.steps_per_launch, &lc.tile_shape) == 7) {
                if (key == k && valid_launch(lc, h->pl)) {
                    fclose(f);
                    lbm_status s = lbm_set_launch(h, &lc);
                    if (s == LBM_OK && chosen) *chosen = h->lc;
                    return s;
                }
            }
            fclose(f);
        }
    }
    const int blocks[] = {128, 256, 512};
    const int npts[] = {1, 2};
    const int xcds[] = {0, 1};
    const int pers[] = {0, 4};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    lbm_launch_config best = h->lc;
    float best_ms = 1e30f;
    const lbm_launch_config saved = h->lc;
    // Every trial reads the live buffer and writes only the other buffer and
    // scratch tallies; times are per step.
    auto trial = [&](const lbm_launch_config &lc, float *ms_per_step) -> lbm_status {
        if (lc.steps_per_launch > 1) {
            lbm_status s = tables_for(h, lc);
            if (s != LBM_OK) return s;
            Step2Launch L = stepk_args(h, lc.steps_per_launch, h->cur, h->acc_scratch(), lc);
            HIP_TRY(launch_stepk(L, h->stream));
            HIP_TRY(hipEventRecord(e0, h->stream));
            for (int k = 0; k < steps; ++k) HIP_TRY(launch_stepk(L, h->stream));
        } else {
            lbm_status s = build_tiles(h, lc);
            if (s != LBM_OK) return s;
            StepLaunch L = step_args(h, 1, h->cur, h->acc_scratch(), 0, (int)h->tiles.size(), lc);
            HIP_TRY(launch_step(L, h->stream));
            HIP_TRY(hipEventRecord(e0, h->stream));
            for (int k = 0; k < steps; ++k) HIP_TRY(launch_step(L, h->stream));
        }
        HIP_TRY(hipEventRecord(e1, h->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        *ms_per_step = ms / (float)(steps * lc.steps_per_launch);
        return LBM_OK;
    };
    // On a failed trial the handle goes back to the shape it had.
    auto abandon = [&](lbm_status s) -> lbm_status {
        const std::string msg = g_err;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)lbm_set_launch(h, &saved);
        return fail(s, "%s", msg.c_str());
    };
    for (int b : blocks)
        for (int np : npts)
            for (int xr : xcds)
                for (int pp : pers) {
                    lbm_launch_config lc{b, np, xr, pp, 1, 0, 0, 0};
                    float ms;
                    lbm_status s = trial(lc, &ms);
                    if (s != LBM_OK) return abandon(s);
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = lc;
                    }
                }
    // multi-step launches: every tile shape, XCD remap on and off, and the
    // persistent grid for the default shape
    const lbm_launch_config one = best;
    for (int kk = 2; kk <= 3; ++kk) {
        if (!has_k(h->pl, kk)) continue;
        for (int shape = 0; shape < LBM_TILE_SHAPES; ++shape)
            for (int xr : xcds)
                for (int pp : pers) {
                    if (shape != 0 && pp != 0) continue;
                    lbm_launch_config lc{one.block, one.nodes_per_thread, xr, pp, kk, shape, 0, 0};
                    float ms;
                    lbm_status s = trial(lc, &ms);
                    if (s != LBM_OK) return abandon(s);
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = lc;
                    }
                }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // The trials wrote the inactive buffer; when the live state is the raw
    // initial state the inactive buffer is not part of the state either.
    lbm_status s = lbm_set_launch(h, &best);
    if (s != LBM_OK) return s;
    if (chosen) *chosen = h->lc;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s %d %d %d %d %d %d\n", key.c_str(), best.block, best.nodes_per_thread, best.xcd_remap,
                    best.persistent, best.steps_per_launch, best.tile_shape);
            fclose(f);
        }
    }
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// Checkpoints
// ---------------------------------------------------------------------------
namespace {
// 02: the split 16-bit forms store their base times the axis weight
// 03: the parameters gain pcm_even_rates
const char kMagic[8] = {'L', 'B', 'M', 'P', 'C', 'M', '0', '3'};

struct CkptHeader {
    char magic[8];
    int32_t prec, n, cur_is_raw, pad;
    int64_t step, nodes, slots;
};
}  // namespace

namespace {
// Checkpoints move device memory through one host buffer of at most this
// many bytes, so saving or loading the largest states needs no host copy of
// the state.
constexpr size_t kCkptChunk = (size_t)64 << 20;

// Device bytes [dev, dev + n) to f, through the host buffer tmp.
bool write_device(FILE *f, const char *dev, size_t n, char *tmp, hipError_t &err) {
    for (size_t o = 0; o < n; o += kCkptChunk) {
        const size_t m = std::min(kCkptChunk, n - o);
        err = hipMemcpy(tmp, dev + o, m, hipMemcpyDeviceToHost);
        if (err != hipSuccess) return false;
        if (fwrite(tmp, 1, m, f) != m) return false;
    }
    return true;
}

// n bytes of f to device memory at dev, through the host buffer tmp.
bool read_device(FILE *f, char *dev, size_t n, char *tmp, hipError_t &err) {
    for (size_t o = 0; o < n; o += kCkptChunk) {
        const size_t m = std::min(kCkptChunk, n - o);
        if (fread(tmp, 1, m, f) != m) return false;
        err = hipMemcpy(dev + o, tmp, m, hipMemcpyHostToDevice);
        if (err != hipSuccess) return false;
    }
    return true;
}

// Bytes of a checkpoint of handle h: header, parameters, initial energy and
// mass, then the state buffer, the source plane and the wall tallies.
int64_t ckpt_bytes(const lbm_handle *h) {
    return (int64_t)sizeof(CkptHeader) + (int64_t)h->n * (sizeof(lbm_params) + 2 * sizeof(double)) +
           h->pl.pop_bytes + h->pl.stride * (int64_t)real_size(h->st) + h->pl.slots * 2 * (int64_t)sizeof(double);
}
}  // namespace

extern "C" lbm_status lbm_save(lbm_handle *h, const char *path) {
    if (!h || !path) return fail(LBM_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(h->stream));
    const size_t sr_bytes = (size_t)h->pl.stride * real_size(h->st);
    std::unique_ptr<char[]> tmp(new (std::nothrow) char[kCkptChunk]);
    if (!tmp) return fail(LBM_ENOMEM, "no host memory for the checkpoint buffer");
    std::vector<double> acc((size_t)h->pl.slots * 2);
    HIP_TRY(hipMemcpy(acc.data(), h->acc(), acc.size() * sizeof(double), hipMemcpyDeviceToHost));
    FILE *f = fopen(path, "wb");
    if (!f) return fail(LBM_EIO, "cannot open %s for writing", path);
    CkptHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    std::memcpy(hd.magic, kMagic, 8);
    hd.prec = (int32_t)h->prec;
    hd.n = h->n;
    hd.cur_is_raw = h->step == 0;
    hd.step = h->step;
    hd.nodes = h->pl.nodes;
    hd.slots = h->pl.slots;
    hipError_t err = hipSuccess;
    bool ok = fwrite(&hd, sizeof(hd), 1, f) == 1;
    ok = ok && fwrite(h->params.data(), sizeof(lbm_params), h->n, f) == (size_t)h->n;
    ok = ok && fwrite(h->E0.data(), sizeof(double), h->n, f) == (size_t)h->n;
    ok = ok && fwrite(h->M0.data(), sizeof(double), h->n, f) == (size_t)h->n;
    ok = ok && write_device(f, (const char *)h->pop(h->cur), (size_t)h->pl.pop_bytes, tmp.get(), err);
    ok = ok && write_device(f, (const char *)h->sr(h->cur), sr_bytes, tmp.get(), err);
    ok = ok && fwrite(acc.data(), sizeof(double), acc.size(), f) == acc.size();
    ok = (fclose(f) == 0) && ok;
    if (err != hipSuccess) return fail(LBM_EDEVICE, "copy of the state for %s: %s", path, hipGetErrorString(err));
    if (!ok) return fail(LBM_EIO, "short write to %s", path);
    return LBM_OK;
}

extern "C" lbm_status lbm_load(lbm_handle *h, const char *path) {
    if (!h || !path) return fail(LBM_EINVAL, "NULL argument");
    FILE *f = fopen(path, "rb");
    if (!f) return fail(LBM_EIO, "cannot open %s", path);
    CkptHeader hd;
    if (fread(&hd, sizeof(hd), 1, f) != 1 || std::memcmp(hd.magic, kMagic, 8) != 0) {
        fclose(f);
        return fail(LBM_EIO, "%s is not a checkpoint of this library", path);
    }
    if (hd.prec != (int32_t)h->prec || hd.n != h->n || hd.nodes != h->pl.nodes || hd.slots != h->pl.slots) {
        fclose(f);
        return fail(LBM_EINVAL, "checkpoint %s was written for other cavities or precision", path);
    }
    std::vector<lbm_params> ps(h->n);
    std::vector<double> E0(h->n), M0(h->n);
    bool ok = fread(ps.data(), sizeof(lbm_params), h->n, f) == (size_t)h->n;
    ok = ok && fread(E0.data(), sizeof(double), h->n, f) == (size_t)h->n;
    ok = ok && fread(M0.data(), sizeof(double), h->n, f) == (size_t)h->n;
    if (!ok) {
        fclose(f);
        return fail(LBM_EIO, "short read from %s", path);
    }
    for (int c = 0; c < h->n; ++c)
        if (std::memcmp(&ps[c], &h->params[c], sizeof(lbm_params)) != 0) {
            fclose(f);
            return fail(LBM_EINVAL, "checkpoint %s: parameters of cavity %d differ", path, c);
        }
    // a file of the wrong length is refused before any device memory changes
    const off_t here = ftello(f);
    if (here < 0 || fseeko(f, 0, SEEK_END) != 0 || ftello(f) != (off_t)ckpt_bytes(h) ||
        fseeko(f, here, SEEK_SET) != 0) {
        fclose(f);
        return fail(LBM_EIO, "%s is not %lld bytes long, as a checkpoint of these cavities is", path,
                    (long long)ckpt_bytes(h));
    }
    std::unique_ptr<char[]> tmp(new (std::nothrow) char[kCkptChunk]);
    if (!tmp) {
        fclose(f);
        return fail(LBM_ENOMEM, "no host memory for the checkpoint buffer");
    }
    // the state goes into the buffer pair the next step would write, and
    // becomes current only once all of it has arrived: a failed load leaves
    // the handle's state as it was
    const hipError_t es = hipStreamSynchronize(h->stream);
    if (es != hipSuccess) {
        fclose(f);
        return fail(LBM_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(es));
    }
    const int nb = 1 - h->cur;
    const size_t sr_bytes = (size_t)h->pl.stride * real_size(h->st);
    std::vector<double> acc((size_t)h->pl.slots * 2);
    hipError_t err = hipSuccess;
    ok = read_device(f, (char *)h->pop(nb), (size_t)h->pl.pop_bytes, tmp.get(), err);
    ok = ok && read_device(f, (char *)h->sr(nb), sr_bytes, tmp.get(), err);
    ok = ok && fread(acc.data(), sizeof(double), acc.size(), f) == acc.size();
    fclose(f);
    if (err != hipSuccess) return fail(LBM_EDEVICE, "copy of the state from %s: %s", path, hipGetErrorString(err));
    if (!ok) return fail(LBM_EIO, "short read from %s", path);
    HIP_TRY(hipMemcpy(h->acc(), acc.data(), acc.size() * sizeof(double), hipMemcpyHostToDevice));
    h->cur = nb;
    h->step = hd.step;
    h->E0 = E0;
    h->M0 = M0;
    return LBM_OK;
}

extern "C" lbm_status lbm_copy_state(lbm_handle *h, int32_t c, void *host, uint64_t bytes) {
    if (!h || !host) return fail(LBM_EINVAL, "NULL argument");
    if (c < 0 || c >= h->n) return fail(LBM_EINVAL, "cavity %d out of range", c);
    const int64_t nn = (int64_t)h->params[c].nx * h->params[c].ny;
    if (bytes < (uint64_t)bytes_per_node(h->st) * nn) return fail(LBM_EINVAL, "host buffer too small");
    HIP_TRY(hipStreamSynchronize(h->stream));
    PlaneGroup grp[2];
    const int ng = plane_groups(h->st, grp);
    const Bands &bd = h->pl.bands[c];
    const int nx = h->params[c].nx, ny = h->params[c].ny;
    const char *blocks = (const char *)h->pop(h->cur) + bd.off;
    char *dst = (char *)host;
    size_t group_off = 0;  // byte offset of the plane group within a block
    for (int q = 0; q < ng; ++q) {
        const size_t eb = grp[q].bytes;
        for (int p = 0; p < grp[q].planes; ++p) {
            // each band's rows of the plane are contiguous in its block
            for (int b = 0; b < bd.count; ++b) {
                const int rows = std::min(bd.rows, ny - b * bd.rows);
                const char *src = blocks + (size_t)b * bd.bytes + group_off + (size_t)p * bd.nodes * eb;
                HIP_TRY(hipMemcpy2D(dst, (size_t)nx * eb, src, (size_t)bd.pitch * eb, (size_t)nx * eb, rows,
                                    hipMemcpyDeviceToHost));
                dst += (size_t)rows * nx * eb;
            }
        }
        group_off += (size_t)grp[q].planes * bd.nodes * eb;
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_debug_poke(lbm_handle *h, int32_t c, int32_t x, int32_t y, int32_t field,
                                     int32_t dir, double value) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (c < 0 || c >= h->n) return fail(LBM_EINVAL, "cavity %d out of range", c);
    const lbm_params &p = h->params[c];
    const int qt = h->pl.lat[c].qt;
    if (x < 0 || x >= p.nx || y < 0 || y >= p.ny || field < 0 || field > 2 || dir < 0 ||
        dir > (field == 0 ? 8 : qt - 1))
        return fail(LBM_EINVAL, "poke index out of range");
    // the node's band block, its index within the band, the plane stride
    const Bands &bd = h->pl.bands[c];
    const int b = y / bd.rows;
    const int64_t node = (int64_t)(y - b * bd.rows) * bd.pitch + x;
    const size_t S = (size_t)bd.nodes;
    char *base = (char *)h->pop(h->cur) + bd.off + (size_t)b * bd.bytes;
    char *ptr;
    int elem;
    if (h->st == ST_F32H || h->st == ST5_F32H) {
        const int nf32 = 8 + 2 * qt;
        if (field == 1 && dir == 0) {
            ptr = base + (size_t)nf32 * S * 4 + (size_t)node * 8;
            elem = 8;
        } else {
            const int plane = field == 0 ? dir : (field == 1 ? 8 + dir : 8 + qt + dir);
            ptr = base + ((size_t)plane * S + node) * 4;
            elem = 4;
        }
    } else if (h->st == ST_F16S || h->st == ST_BF16S) {
        if (dir == 0) {
            ptr = base + ((size_t)(2 * field) * S + node) * 4;
            elem = 4;
        } else {
            ptr = base + (size_t)6 * S * 4 + ((size_t)(8 * field + dir - 1) * S + node) * 2;
            elem = h->st == ST_BF16S ? 3 : 2;
        }
    } else {
        const int eb = bytes_per_node(h->st) / (9 + 2 * qt);
        const int plane = field == 0 ? dir : 9 + (field - 1) * qt + dir;
        ptr = base + ((size_t)plane * S + node) * eb;
        elem = h->st == ST_BF16 ? 3 : eb;
    }
    HIP_TRY(launch_poke(elem, ptr, value, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}
