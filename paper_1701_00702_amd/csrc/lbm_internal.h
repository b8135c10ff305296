// Internal declarations shared by the kernels (lbm_kernels.hip) and the host
// library (lbm_api.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Storage forms.  ST_F64 .. ST_F32H and ST_BF16S carry D2Q9 thermal fields
// (27 populations per node); ST5_* the D2Q5 thermal fields of Appendix B (19).
enum Storage {
    ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3, ST_F16S = 4, ST_F32H = 5,
    ST5_F64 = 6, ST5_F32 = 7, ST5_F32H = 8, ST_BF16S = 9
};

enum Wall { W_LEFT = 0, W_RIGHT = 1, W_BOTTOM = 2, W_TOP = 3 };

// Longest cavity row.  A band (below) holds at least LBM_MIN_BAND_ROWS rows,
// and the step kernels address a tile's rows by 32-bit byte offsets within
// two consecutive bands: band_nodes * (bytes per node + 8) < 2^31.
#define LBM_MAX_NX 262144
#define LBM_MIN_BAND_ROWS 32
// Target size of one band of a state buffer (bytes); a build option.
#ifndef LBM_BAND_BYTES
#define LBM_BAND_BYTES (256ll << 20)
#endif

// Constants of the PCM enthalpy field, kept in both arithmetic types (the
// mixed storage form runs this field in FP64 and the others in FP32).
template <typename T>
struct ThermalConst {
    // enthalpy -> temperature, liquid fraction (Eqs. 38-39)
    T H_fs, H_fl, T_fs, T_fl, inv_dH, dT_band, inv_cps, inv_cpl;
    // equilibrium (Eq. 34 / Eq. B2)
    T c_pl, c_fref, inv_phi;
    // relaxation rates Theta (Eq. 31; D2Q5: the first five in the moment
    // order of Eq. B1) folded with the factors g_k of the inverse transform
    // (D2Q9: 1/|M_k|^2 of Eq. 13; D2Q5: 1, 1/2, 1/2, 1/4, 1/4 of Eq. B1):
    // (1 - zeta_k) g_k and zeta_k g_k
    T zA[9], zB[9];
    // D2Q5: varpi and 1/c_sT^2 = 2/varpi (D2Q9: 1/c_s^2 = 3)
    T varpi, inv_cs2;
    // reference state and the isothermal wall values per wall
    T T_ref, H_ref, T_wall[4], H_wall[4];
};

// Per-cavity constants in the arithmetic type R of the kernels.  One table
// entry per cavity lives in device memory; a workgroup reads the entry of
// its tile through scalar loads.
template <typename R>
struct CavityConst {
    // geometry of the cavity inside the packed node index (the flat
    // per-node arrays of the interstitial source)
    int32_t nx, ny, periodic, gaxis;
    int64_t node0;  // first packed node of this cavity
    int64_t acc0;   // first wall-tally slot of this cavity (2*(nx+ny) slots)
    // Populations are stored by bands: rows [b * band_rows, (b + 1) *
    // band_rows) of the cavity form band b, a block of band_bytes holding
    // every population plane of those rows (node (x, y) at index
    // (y - b * band_rows) * pitch + x of a plane, plane stride band_nodes).
    // The cavity's blocks follow each other from byte pop_off of a state
    // buffer.  Kept to a few hundred MiB, a block keeps the planes a tile
    // reads and writes close together in the address space; the row pitch
    // (nx rounded up to 64 nodes, the padding never read or written) starts
    // every row of every plane on a cache-line boundary.
    int32_t band_rows, pitch;
    int64_t band_nodes, band_bytes, pop_off;
    // materials
    R phi, inv_phi, inv_cpm, c_pm, c_mref;
    // rates folded with the factors of the inverse transform: flow (D2Q9,
    // 1/|M_k|^2 of Eq. 13) (1 - s_k) / |M_k|^2, s_k / |M_k|^2 and the forcing
    // factor (1 - s_k/2) / |M_k|^2; metal (1 - eta_k) g_k, eta_k g_k with the
    // thermal lattice's g_k (D2Q5: 1, 1/2, 1/2, 1/4, 1/4 of Eq. B1)
    R fA[9], fB[9], fC[9], mA[9], mB[9];
    // flow: buoyancy, porous drag, explicit velocity (Eqs. 3, 7, 23-25)
    R gbeta, T0, drag_lin, drag_quad, l0, l0sq, l1;
    // interstitial exchange (Eqs. 36, 47): Sr_f = hv_f (T_m - T_f), Sr_m = hv_m (T_f - T_m)
    R hv_f, hv_m, sr_ratio;  // sr_ratio = hv_m / hv_f
    // reference temperature of the stored offsets; per wall (left, right,
    // bottom, top): isothermal (1) or adiabatic (0) and its temperature
    R T_ref, T_wall[4], varpi;
    int32_t wall_iso[4];
    int32_t bounce_back;  // solid phase: 0 volumetric (Eq. 20), 1 bounce-back (Sec. V B)
    // storage scale per field (populations are stored as (X - X_ref) * scale)
    R scale[3], inv_scale[3];
    // PCM enthalpy field
    ThermalConst<float> tf;
    ThermalConst<double> td;
    // FP64 copies for the energy/mass tallies
    double we, wm;  // phi rho_l and (1 - phi) rho_m
    double g_ref[9], h_ref[9];
    double T_init;
};

// A tile is a run [k0, k1) of one cavity's nodes.  Row tiles (kind 0)
// index the rows 1..ny-2 linearly, k = y * nx + x, and start on 64-node
// boundaries (lanes of row 0 idle); the wall columns are part of their
// rows.  Wall tiles (kind 1) index the bottom and top rows, r in [0, 2 nx),
// each tile within one of the two.  Tiles never straddle cavities.
enum { TILE_INTERIOR = 0, TILE_WALL = 1 };
struct Tile {
    int32_t cav, kind, k0, k1;
};

struct StepLaunch {
    int storage;
    int block, npt, xcd_remap, grid;  // grid: number of workgroups (>= 1)
    int pull;                         // 0: first step, populations are post-streaming already
    const void *src;                  // state buffers (banded population blocks)
    void *dst;
    const void *sr_src;
    void *sr_dst;
    double *acc;                      // wall tallies: [slot][2] (energy, mass)
    const void *cav;                  // CavityConst<R>[]
    const Tile *tiles;
    int ntiles;
};

// A tile of the K-steps-per-launch kernels: w x h nodes of one cavity at
// (x0, y0); no tile starts on the last column or row of its cavity.
struct Tile2 {
    int32_t cav, x0, y0, w, h;
};

struct Step2Launch {
    int storage;
    int steps;  // K: 2 or 3 steps per launch
    int shape;  // tile shape index (0 default; see stepk_tile)
    int grid, xcd_remap;
    const void *src;
    void *dst;
    const void *sr_src;
    void *sr_dst;
    double *acc;
    const void *cav;
    const Tile2 *tiles;
    int ntiles;
};

// Macroscopic fields of rows [y0, y0 + rows) of one cavity.
struct MacroLaunch {
    int storage;
    int raw;  // 1: populations are post-streaming already (step 0)
    int cav_index;
    const void *src;
    const void *cav;     // CavityConst<R>[]
    int y0, rows;
    double *fields;      // 6 planes of rows*nx doubles: ux, uy, T_f, T_m, f_l, rho
};

// Per-block partial sums of the diagnostics kernel.
enum {
    P_FL = 0, P_E, P_M, P_DT, P_U, P_NF,
    P_INE0, P_INE1, P_INE2, P_INE3, P_INM0, P_INM1, P_INM2, P_INM3,
    NPART = 16
};
// Layout of the device-side diagnostics result (doubles).
enum {
    D_FL = 0, D_E, D_M, D_DT, D_U, D_NF, D_NUH, D_NUHP, D_NUC, D_FRONT,
    D_FLUXE = 10, D_FLUXM = 14, NDIAG = 18
};

struct DiagLaunch {
    int nx, ny, periodic;
    int64_t acc0;
    const double *partials;
    int nblocks;
    const double *acc;
    double *out;      // NDIAG doubles
    double L, ke, kf, km, dT;  // kf = phi k_f, km = (1-phi) k_m, ke = kf + km
    // T_f and T_m of the three columns next to each vertical wall, and f_l of
    // the middle row (y = ny / 2): the value at column k (k = 0..5 for
    // x = 0, 1, 2, nx - 3, nx - 2, nx - 1) of row y is tf[y * 6 + k];
    // fl_mid[x] for x in [0, nx).
    const double *tf, *tm, *fl_mid;
};

// Diagnostics without the field planes: a fixed grid of at most
// LBM_DIAG_MAX_BLOCKS workgroups strides over the nodes of one cavity,
// writes per-workgroup partial sums, the wall-column temperatures and the
// middle-row liquid fraction in the compact layout of DiagLaunch.
#define LBM_DIAG_MAX_BLOCKS 2048
struct DiagNodeLaunch {
    int storage;
    int raw;
    int cav_index;
    const void *src;
    const void *cav;
    double *partials;  // [nblocks][NPART]
    int nblocks;       // 1 .. LBM_DIAG_MAX_BLOCKS
    double *tf, *tm;   // [ny][6]
    double *fl_mid;    // [nx]
};

// Initial state of rows [y0, y0 + rows) of one cavity.
struct InitLaunch {
    int storage;
    int cav_index;
    const void *cav;
    void *dst;
    void *sr;
    int y0, rows;
    const double *T_pcm;  // device [rows][nx], may be null
    const double *T_mf;   // device [rows][nx], may be null
};

hipError_t launch_step(const StepLaunch &L, hipStream_t s);
hipError_t launch_stepk(const Step2Launch &L, hipStream_t s);
bool stepk_supported(int storage, int k);  // K steps per launch (K = 2, 3)
// Tile shape `shape` (0 .. LBM_TILE_SHAPES - 1) of the K-step kernel; 0 x 0
// when it does not exist.
#define LBM_TILE_SHAPES 3
void stepk_tile(int storage, int k, int shape, int *tw, int *th);
hipError_t launch_macro(const MacroLaunch &L, int nx, int ny, hipStream_t s);
hipError_t launch_diag(const DiagLaunch &L, int nx, int ny, hipStream_t s);
hipError_t launch_diag_nodes(const DiagNodeLaunch &L, int nx, int ny, hipStream_t s);
int diag_node_blocks(int nx, int ny);  // workgroups of launch_diag_nodes
hipError_t launch_init(const InitLaunch &L, int nx, int ny, hipStream_t s);
hipError_t launch_poke(int elem, void *ptr, double value, hipStream_t s);
int bytes_per_node(int storage);  // stored bytes of one node's populations

}  // namespace lbm
