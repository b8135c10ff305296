// Host-side mapping of a problem description to lattice units and the
// storage plan of the state (bands, tiles), shared by the library
// (lbm_api.hip) and host builds of the per-node arithmetic (the CPU replay
// of the step kernels in the tests).  Host code only.
//
// Mapping (lattice units dx = dt = 1, c_s^2 = 1/3; Eq. 54 and the Sec. IV
// parameter list; rates from Eq. 26, Eq. A19 and Sec. III C).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>

#include "../../include/lbmpcm.h"
#include "lbm_internal.h"

// Record an error message (thread-local, read by lbm_last_error) and
// return st.  Defined once per program (the library: lbm_api.hip).
lbm_status fail(lbm_status st, const char *fmt, ...);

namespace lbm {

struct Lattice {
    int nx, ny, periodic, gaxis;
    int qt;                 // thermal velocities: 9 or 5
    double varpi, cs2T;     // D2Q5 weight parameter, thermal sound speed squared
    double phi, rho_l, rho_m, c_pl, c_ps, c_pm, c_fref, c_mref;
    double L, k_f, k_m, nu_f, nu_e, K, F_phi, gbeta, T0, h_v, L_a, d_p, z;
    double T_fs, T_fl, H_fs, H_fl, T_ref, H_ref;
    double T_hot, T_cold, T_init;
    int wall_type[4];       // resolved: 1 isothermal, 2 adiabatic
    double wall_T[4];
    int solid;              // 0 volumetric (Eq. 20), 1 bounce-back (Sec. V B)
    double zeta_a, eta_a;
    double s[9], zeta[9], eta[9];
    int scale_exp[3];
};

inline double enthalpy_of(const Lattice &l, double T) {
    // inverse of Eq. (38); a tie at the solidus is solid
    if (T <= l.T_fs) return l.c_ps * T;
    if (T >= l.T_fl) return l.c_pl * (T - l.T_fl) + l.H_fl;
    return l.H_fs + (T - l.T_fs) / (l.T_fl - l.T_fs) * (l.H_fl - l.H_fs);
}

// Characteristic length: distance between the walls that carry the imposed
// temperature difference; for the periodic channel, between the no-slip
// walls; or the problem's own.
inline double char_length(const lbm_params &p) {
    if (p.L_char > 0) return p.L_char;
    return p.bc_x == 1 ? p.ny - 1.0 : p.nx - 1.0;
}

// Fewest rows a band may hold: any step-kernel tile (a two-step tile of at
// most 20 rows plus 4 rows of pulls, or a one-step tile of at most 2048
// nodes plus a row of pulls either side) then spans at most two bands.
inline int min_band_rows(int nx) { return std::max(LBM_MIN_BAND_ROWS, (2048 + nx - 1) / nx + 4); }

inline lbm_status map_params(const lbm_params &p, lbm_precision prec, Lattice &l) {
    if (p.nx < 4 || p.ny < 4) return fail(LBM_EINVAL, "grid %dx%d: each side needs >= 4 nodes", p.nx, p.ny);
    // the step kernels address a tile's rows by 32-bit byte offsets from its
    // first row: a few dozen rows of 8-byte elements must stay below 2^31
    if (p.nx > LBM_MAX_NX) return fail(LBM_EINVAL, "grid %dx%d: rows longer than %d nodes", p.nx, p.ny, LBM_MAX_NX);
    if ((int64_t)((p.nx + 63) & ~63) * p.ny >= ((int64_t)1 << 31) - 4096)
        return fail(LBM_EINVAL, "grid %dx%d: rows padded to 64 nodes exceed 2^31 nodes", p.nx, p.ny);
    if (p.band_rows < 0 || (p.band_rows > 0 && p.band_rows < min_band_rows(p.nx) && p.band_rows < p.ny))
        return fail(LBM_EINVAL, "band_rows %d: need 0 or at least %d (or the cavity's %d rows)", p.band_rows,
                    min_band_rows(p.nx), p.ny);
    if ((int64_t)p.nx * p.ny > (int64_t)1 << 31)
        return fail(LBM_EINVAL, "cavity of %dx%d nodes exceeds 2^31 nodes", p.nx, p.ny);
    if (p.bc_x != 0 && p.bc_x != 1) return fail(LBM_EINVAL, "bc_x must be 0 or 1");
    if (p.gravity_axis != 0 && p.gravity_axis != 1) return fail(LBM_EINVAL, "gravity_axis must be 0 or 1");
    if (!(p.porosity > 0.0 && p.porosity < 1.0)) return fail(LBM_EINVAL, "porosity %g not in (0,1)", p.porosity);
    if (!(p.cap_ratio > 0.0)) return fail(LBM_EINVAL, "cap_ratio must be positive");
    if (!(p.k_ratio >= 0.0)) return fail(LBM_EINVAL, "k_ratio must be non-negative");
    if (!(p.Pr > 0.0)) return fail(LBM_EINVAL, "Pr must be positive");
    if (!(p.Ra >= 0.0)) return fail(LBM_EINVAL, "Ra must be non-negative");
    if (!(p.Da > 0.0)) return fail(LBM_EINVAL, "Da must be positive");
    if (!(p.Ste > 0.0)) return fail(LBM_EINVAL, "Ste must be positive");
    if (!(p.Nu_i >= 0.0)) return fail(LBM_EINVAL, "Nu_i must be non-negative");
    if (!(p.T_hot > p.T_cold)) return fail(LBM_EINVAL, "T_hot must exceed T_cold");
    if (!(p.T_liquidus > p.T_solidus)) return fail(LBM_EINVAL, "T_liquidus must exceed T_solidus");
    if (p.thermal_lattice != 0 && p.thermal_lattice != 9 && p.thermal_lattice != 5)
        return fail(LBM_EINVAL, "thermal_lattice must be 9 or 5");
    if (p.thermal_collision != 0 && p.thermal_collision != 1)
        return fail(LBM_EINVAL, "thermal_collision must be 0 (MRT) or 1 (BGK)");
    l.qt = p.thermal_lattice == 5 ? 5 : 9;
    if (l.qt == 5 && prec != LBM_F64 && prec != LBM_F32 && prec != LBM_F32_H64)
        return fail(LBM_EINVAL, "D2Q5 thermal fields are stored as LBM_F64, LBM_F32 or LBM_F32_H64");
    l.varpi = 0.0;
    l.cs2T = 1.0 / 3.0;
    if (l.qt == 5) {
        l.varpi = p.varpi > 0 ? p.varpi : 2.0 / 3.0;
        if (!(l.varpi < 1.0)) return fail(LBM_EINVAL, "varpi %g not in (0,1) (Eq. B2)", p.varpi);
        l.cs2T = 0.5 * l.varpi;
    }
    if (p.thermal_collision == 1 && p.zeta_e > 0)
        return fail(LBM_EINVAL, "zeta_e cannot be set for BGK thermal collisions");
    if (p.pcm_even_rates != 0 && p.pcm_even_rates != 1)
        return fail(LBM_EINVAL, "pcm_even_rates must be 0 or 1");
    if (p.pcm_even_rates == 1 && (p.thermal_collision == 1 || p.thermal_lattice == 5))
        return fail(LBM_EINVAL, "pcm_even_rates applies to D2Q9 MRT thermal fields only");
    if (p.solid_treatment != 0 && p.solid_treatment != 1)
        return fail(LBM_EINVAL, "solid_treatment must be 0 (volumetric, Eq. 20) or 1 (bounce-back, Sec. V B)");
    l.solid = p.solid_treatment;
    for (int w = 0; w < 4; ++w)
        if (p.wall_type[w] < 0 || p.wall_type[w] > 2)
            return fail(LBM_EINVAL, "wall_type[%d] = %d: 0 default, 1 isothermal, 2 adiabatic", w, p.wall_type[w]);
    if (p.bc_x == 1 && (p.wall_type[W_LEFT] != 0 || p.wall_type[W_RIGHT] != 0))
        return fail(LBM_EINVAL, "a periodic-in-x problem has no left or right wall");
    {
        // the cavity of Sec. IV B unless a wall says otherwise
        const int def_t[4] = {p.bc_x == 1 ? 2 : 1, p.bc_x == 1 ? 2 : 1, 2, 2};
        const double def_T[4] = {p.bc_x == 1 ? 0.0 : p.T_hot, p.bc_x == 1 ? 0.0 : p.T_cold, 0.0, 0.0};
        for (int w = 0; w < 4; ++w) {
            l.wall_type[w] = p.wall_type[w] == 0 ? def_t[w] : p.wall_type[w];
            l.wall_T[w] = p.wall_type[w] == 0 ? def_T[w] : (p.wall_type[w] == 1 ? p.wall_T[w] : 0.0);
        }
    }
    l.nx = p.nx;
    l.ny = p.ny;
    l.periodic = p.bc_x;
    l.gaxis = p.gravity_axis;
    l.phi = p.porosity;
    l.rho_l = 1.0;
    l.c_pl = l.c_ps = l.c_pm = 1.0;
    l.rho_m = p.cap_ratio;  // (rho c_p)_m / (rho c_p)_f with unit c_p and rho_l
    l.c_fref = p.cf_ref > 0 ? p.cf_ref : 0.2 * l.c_pl;
    l.c_mref = p.cm_ref > 0 ? p.cm_ref : 1.0 * l.c_pm;
    if (!(l.c_fref < 1.8 * l.c_pl) || !(l.c_mref < 1.8 * l.c_pm))
        return fail(LBM_EINVAL, "reference specific heats must stay below 9/5 c_p (Remark I)");
    const double J = p.J > 0 ? p.J : 1.0;
    l.L = char_length(p);
    const double dpL = p.dp_over_L > 0 ? p.dp_over_L : 0.0135;
    l.d_p = dpL * l.L;
    double kf = p.k_f;
    if (!(kf > 0)) {
        // largest k_f with tau_v, tau_g, tau_h <= 2 and z <= 0.5
        // tau = 0.5 + alpha_ref / c_s^2 <= 2  <=>  alpha_ref <= 1.5 c_s^2
        kf = 0.5 / (J * p.Pr);
        kf = std::min(kf, 1.5 * l.cs2T * l.rho_l * l.c_fref);
        if (p.k_ratio > 0) kf = std::min(kf, 1.5 * l.cs2T * l.rho_m * l.c_mref / p.k_ratio);
        if (p.Nu_i > 0)
            kf = std::min(kf, 0.5 * l.d_p * l.d_p /
                                  (p.Nu_i * (1.0 / (l.phi * l.rho_l * l.c_pl) +
                                             1.0 / ((1.0 - l.phi) * l.rho_m * l.c_pm))));
    }
    l.k_f = kf;
    const double alpha_f = kf / (l.rho_l * l.c_pl);
    l.nu_f = p.Pr * alpha_f;
    l.nu_e = J * l.nu_f;
    l.k_m = p.k_ratio * kf;
    l.h_v = p.Nu_i * kf / (l.d_p * l.d_p);
    l.F_phi = p.F_phi >= 0 ? p.F_phi : 1.75 / std::sqrt(150.0 * l.phi * l.phi * l.phi);
    l.K = p.Da * l.L * l.L;
    const double dT = p.T_hot - p.T_cold;
    l.gbeta = p.Ra * l.nu_f * alpha_f / (dT * l.L * l.L * l.L);
    l.T0 = p.T_cold;
    l.L_a = l.c_pl * dT / p.Ste;
    l.T_fs = p.T_solidus;
    l.T_fl = p.T_liquidus;
    l.H_fs = l.c_ps * l.T_fs;
    l.H_fl = l.c_pl * l.T_fl + l.L_a;
    // reference state of the stored offsets: on D2Q9 the middle of the
    // mushy band; on D2Q5 the initial interior state, whose nodes then hold
    // exact zeros (each measured best for its lattice over a full FP32 run:
    // the D2Q5 rest population otherwise drifts the energy balance)
    if (l.qt == 9) {
        l.T_ref = 0.5 * (l.T_fs + l.T_fl);
        l.H_ref = 0.5 * (l.H_fs + l.H_fl);
    } else {
        l.T_ref = p.T_init;
        l.H_ref = enthalpy_of(l, p.T_init);
    }
    l.T_hot = p.T_hot;
    l.T_cold = p.T_cold;
    l.T_init = p.T_init;
    // relaxation rates: s_v from nu_e (Eq. 26); zeta_alpha, eta_alpha from the
    // reference diffusivities with the thermal lattice's sound speed (Eq. A19
    // and after Eq. 51; App. B); free rates and zeta_e = zeta_eps =
    // 2 - zeta_alpha (Sec. III C, Eq. 53), or the given zeta_e (Sec. V D)
    // for the pair zeta_e = zeta_eps; on request the enthalpy field's stress
    // moments take that rate too instead of zeta_v = 1.2 (pcm_even_rates).
    // D2Q5 rates in the moment order of Eq. (B1), entries 5..8 unused (1).
    // BGK (Sec. V A): every thermal rate 1/tau.
    const double s_v = 1.0 / (0.5 + 3.0 * l.nu_e);
    const double za = 1.0 / (0.5 + kf / (l.rho_l * l.c_fref) / l.cs2T);
    const double ea = 1.0 / (0.5 + l.k_m / (l.rho_m * l.c_mref) / l.cs2T);
    const double ze = p.zeta_e > 0 ? p.zeta_e : 2.0 - za;
    l.zeta_a = za;
    l.eta_a = ea;
    const double s[9] = {1.0, 1.1, 1.1, 1.0, 1.2, 1.0, 1.2, s_v, s_v};
    double zt[9], et[9];
    if (p.thermal_collision == 1) {
        for (int k = 0; k < 9; ++k) {
            zt[k] = k < l.qt ? za : 1.0;
            et[k] = k < l.qt ? ea : 1.0;
        }
    } else if (l.qt == 9) {
        const double zv = p.pcm_even_rates == 1 ? ze : 1.2;
        const double z9[9] = {1.0, ze, ze, za, za, za, za, zv, zv};
        const double e9[9] = {1.0, 1.1, 1.1, ea, ea, ea, ea, 1.2, 1.2};
        for (int k = 0; k < 9; ++k) {
            zt[k] = z9[k];
            et[k] = e9[k];
        }
    } else {
        const double z5[9] = {1.0, za, za, ze, ze, 1.0, 1.0, 1.0, 1.0};
        const double e5[9] = {1.0, ea, ea, 1.1, 1.1, 1.0, 1.0, 1.0, 1.0};
        for (int k = 0; k < 9; ++k) {
            zt[k] = z5[k];
            et[k] = e5[k];
        }
    }
    for (int k = 0; k < 9; ++k) {
        l.s[k] = s[k];
        l.zeta[k] = zt[k];
        l.eta[k] = et[k];
        if (!(s[k] > 0 && s[k] < 2) || !(zt[k] > 0 && zt[k] < 2) || !(et[k] > 0 && et[k] < 2))
            return fail(LBM_EINVAL, "relaxation rate outside (0,2): s_v=%g zeta_a=%g eta_a=%g", s_v, za, ea);
    }
    l.z = l.h_v * (1.0 / (l.phi * l.rho_l * l.c_pl) + 1.0 / ((1.0 - l.phi) * l.rho_m * l.c_pm));
    if (!(l.z < 1.0))
        return fail(LBM_EINVAL, "interstitial exchange number z = %g >= 1: explicit source unstable", l.z);
    // storage scales (16-bit forms): keep the largest expected offset near 2^14
    l.scale_exp[0] = l.scale_exp[1] = l.scale_exp[2] = 0;
    if (prec == LBM_F16_SPLIT || prec == LBM_BF16_SPLIT) {
        // remainders from the rest equilibrium of the base values (small)
        l.scale_exp[0] = 16;
        l.scale_exp[1] = 12;
        l.scale_exp[2] = 12;
    }
    if (prec == LBM_F16_OFFSET) {
        double span_g = 1.0, span_h = 1.0;
        const double Ts[3] = {p.T_hot, p.T_cold, p.T_init};
        for (double T : Ts) {
            span_g = std::max(span_g, std::fabs(enthalpy_of(l, T) - l.H_ref) + std::fabs(T - l.T_ref));
            span_h = std::max(span_h, std::fabs(T - l.T_ref) * l.c_pm);
        }
        l.scale_exp[0] = 16;
        l.scale_exp[1] = std::max(0, std::min(14, (int)std::floor(std::log2(16384.0 / span_g))));
        l.scale_exp[2] = std::max(0, std::min(14, (int)std::floor(std::log2(16384.0 / span_h))));
    }
    return LBM_OK;
}

// 1 / |M_k|^2, the squared norms of the rows of the D2Q9 moment matrix
// (Eq. 13): 9, 36, 36, 6, 12, 6, 12, 4, 4.
inline double row_norm(int k) {
    static const double n2[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};
    return 1.0 / n2[k];
}

// Factors g_k of the thermal lattice's inverse transform: D2Q9 1/|M_k|^2;
// D2Q5 (Eq. B1) 1, 1/2, 1/2, 1/4, 1/4.
inline double thermal_factor(const Lattice &l, int k) {
    static const double g5[5] = {1.0, 0.5, 0.5, 0.25, 0.25};
    return l.qt == 5 ? (k < 5 ? g5[k] : 0.0) : row_norm(k);
}

template <typename T>
ThermalConst<T> make_thermal(const Lattice &l) {
    ThermalConst<T> t;
    std::memset(&t, 0, sizeof(t));
    t.H_fs = (T)l.H_fs;
    t.H_fl = (T)l.H_fl;
    t.T_fs = (T)l.T_fs;
    t.T_fl = (T)l.T_fl;
    t.inv_dH = (T)(1.0 / (l.H_fl - l.H_fs));
    t.dT_band = (T)(l.T_fl - l.T_fs);
    t.inv_cps = (T)(1.0 / l.c_ps);
    t.inv_cpl = (T)(1.0 / l.c_pl);
    t.c_pl = (T)l.c_pl;
    t.c_fref = (T)l.c_fref;
    t.inv_phi = (T)(1.0 / l.phi);
    for (int k = 0; k < 9; ++k) {
        t.zA[k] = (T)((1.0 - l.zeta[k]) * thermal_factor(l, k));
        t.zB[k] = (T)(l.zeta[k] * thermal_factor(l, k));
    }
    t.varpi = (T)l.varpi;
    t.inv_cs2 = (T)(l.qt == 9 ? 3.0 : 2.0 / l.varpi);
    t.T_ref = (T)l.T_ref;
    t.H_ref = (T)l.H_ref;
    for (int w = 0; w < 4; ++w) {
        t.T_wall[w] = (T)l.wall_T[w];
        t.H_wall[w] = (T)enthalpy_of(l, l.wall_T[w]);
    }
    return t;
}

// Banded placement of one cavity's populations in a state buffer.
struct Bands {
    int rows;       // rows per band
    int pitch;      // row pitch: nx rounded up to 64 nodes
    int64_t nodes;  // plane stride within a band (rows * pitch, rounded up)
    int64_t bytes;  // bytes of one band's block
    int64_t off;    // byte offset of the cavity's first block
    int count;      // number of bands
};

// Rows per band: about LBM_BAND_BYTES of state per block (or the rows the
// caller asked for), at least min_band_rows, at most the cavity.  Rows are
// padded to a pitch of 64 nodes and the plane stride is a multiple of 128
// nodes, so every row of every plane starts on a cache-line boundary.
inline Bands bands_of(int nx, int ny, int bpn, int64_t off, int rows_wanted) {
    Bands b;
    b.pitch = (nx + 63) & ~63;
    int64_t rows = LBM_BAND_BYTES / ((int64_t)bpn * b.pitch);
    rows = std::max<int64_t>(rows, min_band_rows(nx));
    if (rows_wanted > 0) rows = rows_wanted;
    b.rows = (int)std::min<int64_t>(rows, ny);
    b.nodes = ((int64_t)b.rows * b.pitch + 127) & ~(int64_t)127;
    b.bytes = (int64_t)bpn * b.nodes;
    b.off = off;
    b.count = (ny + b.rows - 1) / b.rows;
    return b;
}

template <typename R>
CavityConst<R> make_const(const Lattice &l, int64_t node0, int64_t acc0, const Bands &bd) {
    CavityConst<R> c;
    std::memset(&c, 0, sizeof(c));
    c.nx = l.nx;
    c.ny = l.ny;
    c.periodic = l.periodic;
    c.gaxis = l.gaxis;
    c.node0 = node0;
    c.acc0 = acc0;
    c.band_rows = bd.rows;
    c.pitch = bd.pitch;
    c.band_nodes = bd.nodes;
    c.band_bytes = bd.bytes;
    c.pop_off = bd.off;
    c.phi = (R)l.phi;
    c.inv_phi = (R)(1.0 / l.phi);
    c.inv_cpm = (R)(1.0 / l.c_pm);
    c.c_pm = (R)l.c_pm;
    c.c_mref = (R)l.c_mref;
    for (int k = 0; k < 9; ++k) {
        c.fA[k] = (R)((1.0 - l.s[k]) * row_norm(k));
        c.fB[k] = (R)(l.s[k] * row_norm(k));
        c.fC[k] = (R)((1.0 - 0.5 * l.s[k]) * row_norm(k));
        c.mA[k] = (R)((1.0 - l.eta[k]) * thermal_factor(l, k));
        c.mB[k] = (R)(l.eta[k] * thermal_factor(l, k));
    }
    c.gbeta = (R)l.gbeta;
    c.T0 = (R)l.T0;
    const double dl = l.phi * l.nu_f / l.K;             // phi nu_f / K
    const double dq = l.phi * l.F_phi / std::sqrt(l.K);  // phi F_phi / sqrt(K)
    c.drag_lin = (R)dl;
    c.drag_quad = (R)dq;
    const double l0 = 0.5 * (1.0 + 0.5 * dl);          // Eq. (25)
    c.l0 = (R)l0;
    c.l0sq = (R)(l0 * l0);
    c.l1 = (R)(0.5 * dq);
    const double hvf = l.h_v / (l.phi * l.rho_l), hvm = l.h_v / ((1.0 - l.phi) * l.rho_m);
    c.hv_f = (R)hvf;
    c.hv_m = (R)hvm;
    c.sr_ratio = (R)((l.phi * l.rho_l) / ((1.0 - l.phi) * l.rho_m));
    c.T_ref = (R)l.T_ref;
    c.varpi = (R)l.varpi;
    for (int w = 0; w < 4; ++w) {
        c.T_wall[w] = (R)l.wall_T[w];
        c.wall_iso[w] = l.wall_type[w] == 1 ? 1 : 0;
    }
    c.bounce_back = l.solid;
    for (int f = 0; f < 3; ++f) {
        c.scale[f] = (R)std::ldexp(1.0, l.scale_exp[f]);
        c.inv_scale[f] = (R)std::ldexp(1.0, -l.scale_exp[f]);
    }
    c.tf = make_thermal<float>(l);
    c.td = make_thermal<double>(l);
    c.we = l.phi * l.rho_l;
    c.wm = (1.0 - l.phi) * l.rho_m;
    // reference equilibria at rest (Eqs. 40, 49 / Eqs. B3, B5)
    const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const double wrest = l.qt == 9 ? 5.0 / 9.0 : l.varpi;
    for (int i = 0; i < 9; ++i) {
        const double wi = l.qt == 9 ? w[i] : (i < 5 ? 0.25 * l.varpi : 0.0);
        c.g_ref[i] = i == 0 ? l.H_ref - wrest * l.c_fref * l.T_ref : wi * l.c_fref * l.T_ref;
        c.h_ref[i] = i == 0 ? (l.c_pm - wrest * l.c_mref) * l.T_ref : wi * l.c_mref * l.T_ref;
    }
    c.T_init = l.T_init;
    return c;
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Copy of a parameter struct with its trailing padding cleared, so that
// checkpoints compare parameters byte for byte.
inline lbm_params normalized(const lbm_params &p) {
    lbm_params q = p;
    const size_t end = offsetof(lbm_params, band_rows) + sizeof(q.band_rows);
    std::memset((char *)&q + end, 0, sizeof(q) - end);
    return q;
}

inline int storage_of(lbm_precision p, int qt = 9) {
    if (qt == 5) {
        switch (p) {
            case LBM_F64: return ST5_F64;
            case LBM_F32: return ST5_F32;
            case LBM_F32_H64: return ST5_F32H;
            default: return -1;
        }
    }
    switch (p) {
        case LBM_F64: return ST_F64;
        case LBM_F32: return ST_F32;
        case LBM_F16_OFFSET: return ST_F16;
        case LBM_BF16_OFFSET: return ST_BF16;
        case LBM_F16_SPLIT: return ST_F16S;
        case LBM_BF16_SPLIT: return ST_BF16S;
        case LBM_F32_H64: return ST_F32H;
    }
    return -1;
}

inline size_t real_size(int st) { return (st == ST_F64 || st == ST5_F64) ? 8 : 4; }

// Plane groups of one buffer: {number of planes, bytes per element}.
struct PlaneGroup {
    int planes, bytes;
};
inline int plane_groups(int st, PlaneGroup g[2]) {
    switch (st) {
        case ST_F64: g[0] = {27, 8}; return 1;
        case ST_F32: g[0] = {27, 4}; return 1;
        case ST_F16:
        case ST_BF16: g[0] = {27, 2}; return 1;
        case ST_F16S:
        case ST_BF16S: g[0] = {6, 4}; g[1] = {24, 2}; return 2;
        case ST_F32H: g[0] = {26, 4}; g[1] = {1, 8}; return 2;
        case ST5_F64: g[0] = {19, 8}; return 1;
        case ST5_F32: g[0] = {19, 4}; return 1;
        case ST5_F32H: g[0] = {18, 4}; g[1] = {1, 8}; return 2;
    }
    return 0;
}

// Splits [0, n) into runs of at most t (t >= 3, n >= 4) such that no run
// starts at n - 1: a last run of one would leave a wall node whose partner
// pulls from outside the K-step kernels' LDS region.
inline void split_runs(int n, int t, std::vector<std::pair<int, int>> &out) {
    out.clear();
    if (t < 2) return;
    int start = 0;
    while (start < n) {
        int w = std::min(t, n - start);
        if (n - (start + w) == 1) w -= 1;
        out.push_back({start, w});
        start += w;
    }
}

// Tiles of the K-step kernels for one cavity, row by row (ordering them in
// narrow vertical strips measured no different).
inline void cavity_tiles2(int cav, int nx, int ny, int tw, int th, std::vector<Tile2> &tiles) {
    std::vector<std::pair<int, int>> xs, ys;
    split_runs(nx, tw, xs);
    split_runs(ny, th, ys);
    for (const auto &yr : ys)
        for (const auto &xr : xs) tiles.push_back(Tile2{cav, xr.first, yr.first, xr.second, yr.second});
}

inline int64_t count_tiles2(int nx, int ny, int tw, int th) {
    std::vector<std::pair<int, int>> xs, ys;
    split_runs(nx, tw, xs);
    split_runs(ny, th, ys);
    return (int64_t)xs.size() * (int64_t)ys.size();
}

}  // namespace lbm
