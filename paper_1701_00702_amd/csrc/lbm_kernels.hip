// Device code for the enthalpy-based MRT lattice Boltzmann method for
// solid-liquid phase change in metal foams under local thermal
// non-equilibrium (Liu, He & Li, arXiv:1701.00702), written for gfx950.
//
// One launch of step_kernel advances every node of every cavity by one time
// step.  Per node (one thread per node, pull streaming, structure-of-arrays
// planes, A/B buffers):
//   1. pull the 27 post-collision populations of the neighbours (Eqs. 15, 33,
//      44); a wall node instead pulls the populations of its interior partner
//      and rebuilds its own by non-equilibrium extrapolation (Eq. 52 and its
//      thermal analogues);
//   2. H (Eq. 37), T_f and f_l without iteration (Eqs. 38-39), T_m (Eq. 48),
//      rho (Eq. 21), the volumetric blend with the solid at rest (Eq. 20),
//      buoyancy (Eq. 7), explicit velocity (Eqs. 23-25), total force (Eq. 3);
//   3. the flow collision in moment space with forcing (Eqs. 14, 16-19);
//   4. interstitial sources with the backward-difference time derivative
//      (Eqs. 36, 47, Remark III);
//   5. the enthalpy and metal-foam collisions (Eqs. 32, 34-35; 43, 45-46);
//   6. store the 27 post-collision populations and the source, and tally the
//      energy/mass carried across wall links (FP64, one slot per
//      wall-adjacent node, no atomics).
// The 9x9 transforms are expanded by hand (entries 0, +-1, +-2, +-4) and the
// work stays on the vector ALUs: with roughly two flops per byte the step is
// bound by HBM bandwidth, not by matrix throughput.
//
// Populations are stored as offsets from a fixed reference equilibrium
// (flow: w_i rho_0; enthalpy/metal: the equilibria at the middle of the
// mushy band), times a power-of-two scale for the 16-bit forms.  The moment
// algebra is affine, so the whole update runs on the offsets; the FP32 form
// then keeps the small momentum of the Darcy-scale flow out of the rounding
// of O(1) populations.

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "lbm_internal.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Lattice (Eq. 11) and weights.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int ex_of(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey_of(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
template <typename R>
__host__ __device__ constexpr R w_of(int i) {
    return i == 0 ? R(4) / R(9) : (i <= 4 ? R(1) / R(9) : R(1) / R(36));
}

// ---------------------------------------------------------------------------
// Storage codecs: value in registers = stored * inv_scale (offset form).
// ---------------------------------------------------------------------------
template <typename S>
struct Codec;
template <>
struct Codec<double> {
    static constexpr bool scaled = false;
    __device__ static double load(const double *p, int64_t i) { return __builtin_nontemporal_load(p + i); }
    __device__ static void store(double *p, int64_t i, double v) { __builtin_nontemporal_store(v, p + i); }
    __device__ static double from_double(double v) { return v; }
};
template <>
struct Codec<float> {
    static constexpr bool scaled = false;
    __device__ static float load(const float *p, int64_t i) { return __builtin_nontemporal_load(p + i); }
    __device__ static void store(float *p, int64_t i, float v) { __builtin_nontemporal_store(v, p + i); }
    __device__ static float from_double(double v) { return (float)v; }
};
template <>
struct Codec<__half> {
    static constexpr bool scaled = true;
    __device__ static float load(const __half *p, int64_t i) {
        unsigned short b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p) + i);
        return __half2float(__ushort_as_half(b));
    }
    __device__ static void store(__half *p, int64_t i, float v) {
        unsigned short b = __half_as_ushort(__float2half_rn(v));
        __builtin_nontemporal_store(b, reinterpret_cast<unsigned short *>(p) + i);
    }
    __device__ static __half from_double(double v) { return __float2half_rn((float)v); }
};
template <>
struct Codec<__hip_bfloat16> {
    static constexpr bool scaled = true;
    __device__ static float load(const __hip_bfloat16 *p, int64_t i) {
        unsigned short b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p) + i);
        return __uint_as_float(((unsigned int)b) << 16);
    }
    __device__ static void store(__hip_bfloat16 *p, int64_t i, float v) {
        // round to nearest even on the top 16 bits (finite inputs)
        unsigned int u = __float_as_uint(v);
        u += 0x7fffu + ((u >> 16) & 1u);
        unsigned short b = (unsigned short)(u >> 16);
        __builtin_nontemporal_store(b, reinterpret_cast<unsigned short *>(p) + i);
    }
    __device__ static __hip_bfloat16 from_double(double v) { return __float2bfloat16((float)v); }
};

template <typename S>
struct RealOf {
    using type = float;
};
template <>
struct RealOf<double> {
    using type = double;
};

// ---------------------------------------------------------------------------
// Moment transforms of Eq. (13) on offsets.  d = M q and q = M^-1 d with
// M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void to_moments(const R q[9], R d[9]) {
    const R s14 = (q[1] + q[2]) + (q[3] + q[4]);
    const R s58 = (q[5] + q[6]) + (q[7] + q[8]);
    d[0] = q[0] + s14 + s58;
    d[1] = -R(4) * q[0] - s14 + R(2) * s58;
    d[2] = R(4) * q[0] - R(2) * s14 + s58;
    const R dxd = (q[5] - q[6]) - (q[7] - q[8]);
    const R dyd = (q[5] + q[6]) - (q[7] + q[8]);
    d[3] = (q[1] - q[3]) + dxd;
    d[4] = R(2) * (q[3] - q[1]) + dxd;
    d[5] = (q[2] - q[4]) + dyd;
    d[6] = R(2) * (q[4] - q[2]) + dyd;
    d[7] = (q[1] + q[3]) - (q[2] + q[4]);
    d[8] = (q[5] + q[7]) - (q[6] + q[8]);
}

template <typename R>
__device__ __forceinline__ void from_moments(const R d[9], R q[9]) {
    const R a0 = d[0] * (R(1) / R(9));
    const R a1 = d[1] * (R(1) / R(36));
    const R a2 = d[2] * (R(1) / R(36));
    const R a3 = d[3] * (R(1) / R(6));
    const R a4 = d[4] * (R(1) / R(12));
    const R a5 = d[5] * (R(1) / R(6));
    const R a6 = d[6] * (R(1) / R(12));
    const R a7 = d[7] * R(0.25);
    const R a8 = d[8] * R(0.25);
    const R axis = a0 - a1 - R(2) * a2;
    const R diag = a0 + R(2) * a1 + a2;
    const R xa = a3 - R(2) * a4, ya = a5 - R(2) * a6;
    const R xd = a3 + a4, yd = a5 + a6;
    q[0] = a0 - R(4) * a1 + R(4) * a2;
    q[1] = axis + xa + a7;
    q[2] = axis + ya - a7;
    q[3] = axis - xa + a7;
    q[4] = axis - ya - a7;
    q[5] = diag + xd + yd + a8;
    q[6] = diag - xd + yd - a8;
    q[7] = diag - xd - yd + a8;
    q[8] = diag + xd - yd - a8;
}

// ---------------------------------------------------------------------------
// Macroscopic values of one node from its post-streaming offsets.
// ---------------------------------------------------------------------------
template <typename R>
struct Macro {
    R dH, H, Tf, fl, dTm, Tm, drho, rho, ux, uy, Gx, Gy;
};

// Eqs. (38)-(39), branches in the order the paper lists them.
template <typename R>
__device__ __forceinline__ void eos(const CavityConst<R> &c, R H, R &T, R &fl) {
    if (H <= c.H_fs) {
        T = H * c.inv_cps;
        fl = R(0);
    } else if (H >= c.H_fl) {
        T = c.T_fl + (H - c.H_fl) * c.inv_cpl;
        fl = R(1);
    } else {
        fl = (H - c.H_fs) * c.inv_dH;
        T = c.T_fs + fl * c.dT_band;
    }
}

// Blends qf in place (Eq. 20) and computes everything the collisions need.
template <typename R>
__device__ __forceinline__ void macros(const CavityConst<R> &c, R qf[9], const R qg[9],
                                       const R qh[9], Macro<R> &m) {
    m.dH = ((qg[0] + qg[1]) + (qg[2] + qg[3])) + ((qg[4] + qg[5]) + (qg[6] + qg[7])) + qg[8];
    m.H = c.H_ref + m.dH;
    eos(c, m.H, m.Tf, m.fl);
    const R dE = ((qh[0] + qh[1]) + (qh[2] + qh[3])) + ((qh[4] + qh[5]) + (qh[6] + qh[7])) + qh[8];
    m.dTm = dE * c.inv_cpm;
    m.Tm = c.T_ref + m.dTm;
    m.drho = ((qf[0] + qf[1]) + (qf[2] + qf[3])) + ((qf[4] + qf[5]) + (qf[6] + qf[7])) + qf[8];
    m.rho = R(1) + m.drho;
    // Eq. (20): f = f_l f+ + (1 - f_l) w rho, written on offsets from w rho_0.
    const R sol = (R(1) - m.fl) * m.drho;
#pragma unroll
    for (int i = 0; i < 9; ++i) qf[i] = m.fl * qf[i] + w_of<R>(i) * sol;
    // Eq. (7): buoyancy along +axis (gravity along -axis).
    const R G = c.gbeta * (m.Tf - c.T0) * m.fl;
    m.Gx = c.gaxis == 0 ? G : R(0);
    m.Gy = c.gaxis == 1 ? G : R(0);
    // Eq. (24), Eq. (23).
    const R jx = (qf[1] - qf[3]) + ((qf[5] - qf[6]) - (qf[7] - qf[8]));
    const R jy = (qf[2] - qf[4]) + ((qf[5] + qf[6]) - (qf[7] + qf[8]));
    const R inv_rho = R(1) / m.rho;
    const R vx = jx * inv_rho + R(0.5) * c.phi * m.Gx;
    const R vy = jy * inv_rho + R(0.5) * c.phi * m.Gy;
    const R vmag = sqrt(vx * vx + vy * vy);
    const R inv_den = R(1) / (c.l0 + sqrt(c.l0sq + c.l1 * vmag));
    m.ux = vx * inv_den;
    m.uy = vy * inv_den;
}

// Flow collision, Eqs. (14), (16)-(19), on the blended offsets.
template <typename R>
__device__ __forceinline__ void collide_flow(const CavityConst<R> &c, const Macro<R> &m, R q[9]) {
    R d[9];
    to_moments(q, d);
    const R ux = m.ux, uy = m.uy, rho = m.rho;
    const R uu = ux * ux + uy * uy;
    const R umag = sqrt(uu);
    // Eq. (3).
    const R Fx = -c.drag_lin * ux - c.drag_quad * umag * ux + c.phi * m.Gx;
    const R Fy = -c.drag_lin * uy - c.drag_quad * umag * uy + c.phi * m.Gy;
    const R rip = rho * c.inv_phi;
    R eq[9], S[9];
    eq[1] = -R(2) * m.drho + R(3) * rip * uu;
    eq[2] = m.drho - R(3) * rip * uu;
    eq[3] = rho * ux;
    eq[4] = -eq[3];
    eq[5] = rho * uy;
    eq[6] = -eq[5];
    eq[7] = rip * (ux * ux - uy * uy);
    eq[8] = rip * ux * uy;
    const R uF = ux * Fx + uy * Fy;
    S[1] = R(6) * rip * uF;
    S[2] = -S[1];
    S[3] = rho * Fx;
    S[4] = -S[3];
    S[5] = rho * Fy;
    S[6] = -S[5];
    S[7] = R(2) * rip * (ux * Fx - uy * Fy);
    S[8] = rip * (ux * Fy + uy * Fx);
    d[0] = m.drho;
#pragma unroll
    for (int k = 1; k < 9; ++k) d[k] = d[k] - c.s[k] * (d[k] - eq[k]) + c.s_half[k] * S[k];
    from_moments(d, q);
}

// PCM enthalpy collision, Eqs. (32), (34)-(35).
template <typename R>
__device__ __forceinline__ void collide_pcm(const CavityConst<R> &c, const Macro<R> &m, R S_pcm,
                                            R q[9]) {
    R d[9];
    to_moments(q, d);
    const R dT = m.Tf - c.T_ref;
    const R jT = c.c_pl * m.Tf * c.inv_phi;
    R eq[9];
    eq[0] = m.dH;
    eq[1] = -R(4) * m.dH + R(2) * c.c_fref * dT;
    eq[2] = R(4) * m.dH - R(3) * c.c_fref * dT;
    eq[3] = jT * m.ux;
    eq[4] = -eq[3];
    eq[5] = jT * m.uy;
    eq[6] = -eq[5];
    eq[7] = R(0);
    eq[8] = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = d[k] - c.zeta[k] * (d[k] - eq[k]);
    d[0] += S_pcm;
    d[1] -= R(2) * S_pcm;
    d[2] += S_pcm;
    from_moments(d, q);
}

// Metal-foam collision, Eqs. (43), (45)-(46).
template <typename R>
__device__ __forceinline__ void collide_metal(const CavityConst<R> &c, const Macro<R> &m,
                                              R S_metal, R q[9]) {
    R d[9];
    to_moments(q, d);
    const R e = c.c_pm * m.dTm;
    R eq[9];
    eq[0] = e;
    eq[1] = (-R(4) * c.c_pm + R(2) * c.c_mref) * m.dTm;
    eq[2] = (R(4) * c.c_pm - R(3) * c.c_mref) * m.dTm;
#pragma unroll
    for (int k = 3; k < 9; ++k) eq[k] = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = d[k] - c.eta[k] * (d[k] - eq[k]);
    d[0] += S_metal;
    d[1] -= R(2) * S_metal;
    d[2] += S_metal;
    from_moments(d, q);
}

// Non-equilibrium extrapolation for wall node (x, y), applied to the
// partner's pulled offsets in place (Eq. 52 with wall velocity 0; thermal
// analogues with the isothermal or zero-gradient wall values).
template <typename R>
__device__ __forceinline__ void reconstruct_wall(const CavityConst<R> &c, int x, R qf[9], R qg[9],
                                                 R qh[9]) {
    R tf[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) tf[i] = qf[i];
    Macro<R> p;
    macros(c, tf, qg, qh, p);
    R Tb, Hb, Tmb;
    const bool vertical = !c.periodic && (x == 0 || x == c.nx - 1);
    if (vertical) {
        const bool hot = (x == 0);
        Tb = hot ? c.T_hot : c.T_cold;
        Hb = hot ? c.H_hot : c.H_cold;
        Tmb = Tb;
    } else {
        Tb = p.Tf;
        Hb = p.H;
        Tmb = p.Tm;
    }
    const R uu = p.ux * p.ux + p.uy * p.uy;
    const R dTg = Tb - p.Tf;
    const R dTh = Tmb - p.Tm;
    const R jT = R(3) * c.c_pl * p.Tf * c.inv_phi;
    qf[0] += -w_of<R>(0) * p.rho * (-R(1.5) * uu * c.inv_phi);
    qg[0] += (Hb - p.H) - R(5) / R(9) * c.c_fref * dTg;
    qh[0] += (c.c_pm - R(5) / R(9) * c.c_mref) * dTh;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const R eu = R(ex_of(i)) * p.ux + R(ey_of(i)) * p.uy;
        // f^eq(rho, 0) - f^eq(rho, u) from Eq. (27)
        qf[i] += -w_of<R>(i) * p.rho * (R(3) * eu + R(4.5) * eu * eu * c.inv_phi - R(1.5) * uu * c.inv_phi);
        // g^eq(H_b, T_b, 0) - g^eq(H, T, u) from Eq. (40)
        qg[i] += w_of<R>(i) * (c.c_fref * dTg - jT * eu);
        // h^eq(T_mb) - h^eq(T_m) from Eq. (49)
        qh[i] += w_of<R>(i) * c.c_mref * dTh;
    }
}

// ---------------------------------------------------------------------------
// The fused step kernel.
// ---------------------------------------------------------------------------
template <typename S>
struct Planes {
    const S *__restrict__ src;
    S *__restrict__ dst;
    int64_t stride;
};

template <typename S, typename R, bool PULL>
__device__ __forceinline__ void step_node(const CavityConst<R> &c, const S *__restrict__ src,
                                          S *__restrict__ dst, int64_t stride,
                                          const R *__restrict__ sr_src, R *__restrict__ sr_dst,
                                          double *__restrict__ acc, int x, int y) {
    using C = Codec<S>;
    const int nx = c.nx, ny = c.ny;
    const int64_t n0 = c.node0;
    const int own = y * nx + x;
    const bool vwall = !c.periodic && (x == 0 || x == nx - 1);
    const bool hwall = (y == 0 || y == ny - 1);
    const bool wall = vwall || hwall;
    int sx = x, sy = y;
    if (PULL && wall) {
        if (!c.periodic) sx = (x == 0) ? 1 : ((x == nx - 1) ? nx - 2 : x);
        sy = (y == 0) ? 1 : ((y == ny - 1) ? ny - 2 : y);
    }

    R qf[9], qg[9], qh[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int idx = own;
        if (PULL) {
            int px = sx - ex_of(i);
            if (c.periodic) px = px < 0 ? px + nx : (px >= nx ? px - nx : px);
            idx = (sy - ey_of(i)) * nx + px;
        }
        const int64_t k = n0 + idx;
        qf[i] = (R)C::load(src + (int64_t)i * stride, k);
        qg[i] = (R)C::load(src + (int64_t)(9 + i) * stride, k);
        qh[i] = (R)C::load(src + (int64_t)(18 + i) * stride, k);
    }
    if (C::scaled) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            qf[i] *= c.inv_scale[0];
            qg[i] *= c.inv_scale[1];
            qh[i] *= c.inv_scale[2];
        }
    }
    const R sr_prev = sr_src[n0 + own];

    // Wall tallies: interior nodes next to a wall own one slot per wall they
    // touch.  xw: the vertical wall (x = 1 or nx-2), yw: the horizontal one.
    const bool near_x = !wall && !c.periodic && (x == 1 || x == nx - 2);
    const bool near_y = !wall && (y == 1 || y == ny - 2);
    double xE = 0.0, xM = 0.0, yE = 0.0, yM = 0.0;
    if (PULL && (near_x || near_y)) {
        // inflow: populations pulled from wall nodes (post-collision of the
        // previous step)
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int px = x - ex_of(i), py = y - ey_of(i);
            const bool onx = !c.periodic && (px == 0 || px == nx - 1);
            const bool ony = (py == 0 || py == ny - 1);
            if (onx || ony) {
                const double e = c.we * (c.g_ref[i] + (double)qg[i]) + c.wm * (c.h_ref[i] + (double)qh[i]);
                const double mm = (double)w_of<double>(i) + (double)qf[i];
                if (onx) {
                    xE += e;
                    xM += mm;
                } else {
                    yE += e;
                    yM += mm;
                }
            }
        }
    }

    if (PULL && wall) reconstruct_wall(c, x, qf, qg, qh);

    Macro<R> m;
    macros(c, qf, qg, qh, m);
    collide_flow(c, m, qf);
    // Eqs. (36), (47) with the backward difference of Remark III.
    const R srf = c.hv_f * (m.Tm - m.Tf);
    const R srm = c.hv_m * (m.Tf - m.Tm);
    const R srm_prev = -c.sr_ratio * sr_prev;
    const R S_pcm = srf + R(0.5) * (srf - sr_prev);
    const R S_metal = srm + R(0.5) * (srm - srm_prev);
    collide_pcm(c, m, S_pcm, qg);
    collide_metal(c, m, S_metal, qh);

    if (near_x || near_y) {
        // outflow: post-collision populations aimed at wall nodes
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int tx = x + ex_of(i), ty = y + ey_of(i);
            const bool onx = !c.periodic && (tx == 0 || tx == nx - 1);
            const bool ony = (ty == 0 || ty == ny - 1);
            if (onx || ony) {
                const double e = c.we * (c.g_ref[i] + (double)qg[i]) + c.wm * (c.h_ref[i] + (double)qh[i]);
                const double mm = (double)w_of<double>(i) + (double)qf[i];
                if (onx) {
                    xE -= e;
                    xM -= mm;
                } else {
                    yE -= e;
                    yM -= mm;
                }
            }
        }
        if (near_x) {
            const int64_t slot = c.acc0 + (x == 1 ? y : ny + y);
            acc[2 * slot] += xE;
            acc[2 * slot + 1] += xM;
        }
        if (near_y) {
            const int64_t slot = c.acc0 + 2 * ny + (y == 1 ? x : nx + x);
            acc[2 * slot] += yE;
            acc[2 * slot + 1] += yM;
        }
    }

    const int64_t k = n0 + own;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        R a = qf[i], b = qg[i], d = qh[i];
        if (C::scaled) {
            a *= c.scale[0];
            b *= c.scale[1];
            d *= c.scale[2];
        }
        C::store(dst + (int64_t)i * stride, k, a);
        C::store(dst + (int64_t)(9 + i) * stride, k, b);
        C::store(dst + (int64_t)(18 + i) * stride, k, d);
    }
    sr_dst[k] = srf;
}

__device__ __forceinline__ int remap_block(int b, int grid, int xcd_remap) {
    // Hardware hands consecutive workgroups to the 8 XCDs in turn; this maps
    // them back so that each XCD walks a contiguous range of tiles.
    if (!xcd_remap) return b;
    const int full = grid & ~7;
    if (b >= full) return b;
    const int per = full >> 3;
    return (b & 7) * per + (b >> 3);
}

template <typename S, typename R, bool PULL, int NPT>
__global__ __launch_bounds__(512) void step_kernel(const S *__restrict__ src, S *__restrict__ dst,
                                                   int64_t stride, const R *__restrict__ sr_src,
                                                   R *__restrict__ sr_dst, double *__restrict__ acc,
                                                   const CavityConst<R> *__restrict__ cav,
                                                   const Tile *__restrict__ tiles, int ntiles,
                                                   int xcd_remap) {
    const int b = remap_block(blockIdx.x, gridDim.x, xcd_remap);
    for (int t = b; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const CavityConst<R> &c = cav[tl.cav];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int x = tl.x0 + (int)threadIdx.x + j * (int)blockDim.x;
            if (x < tl.x1) step_node<S, R, PULL>(c, src, dst, stride, sr_src, sr_dst, acc, x, tl.y);
        }
    }
}

template <typename S, bool PULL, int NPT>
static hipError_t launch_step_t(const StepLaunch &L, hipStream_t s) {
    using R = typename RealOf<S>::type;
    hipLaunchKernelGGL((step_kernel<S, R, PULL, NPT>), dim3(L.grid), dim3(L.block), 0, s,
                       (const S *)L.src, (S *)L.dst, L.plane_stride, (const R *)L.sr_src,
                       (R *)L.sr_dst, L.acc, (const CavityConst<R> *)L.cav, L.tiles, L.ntiles,
                       L.xcd_remap);
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_step_s(const StepLaunch &L, hipStream_t s) {
    if (!L.pull) return launch_step_t<S, false, 1>(L, s);
    switch (L.npt) {
        case 1: return launch_step_t<S, true, 1>(L, s);
        case 2: return launch_step_t<S, true, 2>(L, s);
        case 4: return launch_step_t<S, true, 4>(L, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(const StepLaunch &L, hipStream_t s) {
    if (L.block < 64 || L.block > 512 || (L.block & 63) || L.grid < 1 || L.ntiles < 1)
        return hipErrorInvalidValue;
    switch (L.storage) {
        case ST_F64: return launch_step_s<double>(L, s);
        case ST_F32: return launch_step_s<float>(L, s);
        case ST_F16: return launch_step_s<__half>(L, s);
        case ST_BF16: return launch_step_s<__hip_bfloat16>(L, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Macroscopic fields and per-block diagnostics of one cavity.
// ---------------------------------------------------------------------------
constexpr int MB = 256;  // threads per block of the diagnostics kernels

int macro_blocks(int nx, int ny) { return (int)(((int64_t)nx * ny + MB - 1) / MB); }

template <typename S, typename R>
__global__ __launch_bounds__(MB) void macro_kernel(const S *__restrict__ src, int64_t stride,
                                                   const CavityConst<R> *__restrict__ cav, int ci,
                                                   int raw, double *__restrict__ fields,
                                                   double *__restrict__ partials) {
    using C = Codec<S>;
    const CavityConst<R> &c = cav[ci];
    const int nx = c.nx, ny = c.ny;
    const int64_t nn = (int64_t)nx * ny;
    const int64_t kk = (int64_t)blockIdx.x * MB + threadIdx.x;
    double v[NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k) v[k] = 0.0;
    if (kk < nn) {
        const int x = (int)(kk % nx), y = (int)(kk / nx);
        const bool vwall = !c.periodic && (x == 0 || x == nx - 1);
        const bool hwall = (y == 0 || y == ny - 1);
        const bool wall = vwall || hwall;
        int sx = x, sy = y;
        if (!raw && wall) {
            if (!c.periodic) sx = (x == 0) ? 1 : ((x == nx - 1) ? nx - 2 : x);
            sy = (y == 0) ? 1 : ((y == ny - 1) ? ny - 2 : y);
        }
        R qf[9], qg[9], qh[9];
        bool finite = true;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int idx = y * nx + x;
            if (!raw) {
                int px = sx - ex_of(i);
                if (c.periodic) px = px < 0 ? px + nx : (px >= nx ? px - nx : px);
                idx = (sy - ey_of(i)) * nx + px;
            }
            const int64_t k = c.node0 + idx;
            qf[i] = (R)C::load(src + (int64_t)i * stride, k) * c.inv_scale[0];
            qg[i] = (R)C::load(src + (int64_t)(9 + i) * stride, k) * c.inv_scale[1];
            qh[i] = (R)C::load(src + (int64_t)(18 + i) * stride, k) * c.inv_scale[2];
            finite = finite && isfinite(qf[i]) && isfinite(qg[i]) && isfinite(qh[i]);
        }
        // inflow of the last step through the wall links (not yet tallied)
        if (!raw && !wall) {
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const int px = x - ex_of(i), py = y - ey_of(i);
                const bool onx = !c.periodic && (px == 0 || px == nx - 1);
                const bool ony = (py == 0 || py == ny - 1);
                if (onx || ony) {
                    const int w = onx ? (px == 0 ? W_LEFT : W_RIGHT) : (py == 0 ? W_BOTTOM : W_TOP);
                    const double e = c.we * (c.g_ref[i] + (double)qg[i]) + c.wm * (c.h_ref[i] + (double)qh[i]);
                    const double mm = (double)w_of<double>(i) + (double)qf[i];
                    // unrolled selects keep the accumulators in registers
                    v[P_INE0] += w == 0 ? e : 0.0;
                    v[P_INE1] += w == 1 ? e : 0.0;
                    v[P_INE2] += w == 2 ? e : 0.0;
                    v[P_INE3] += w == 3 ? e : 0.0;
                    v[P_INM0] += w == 0 ? mm : 0.0;
                    v[P_INM1] += w == 1 ? mm : 0.0;
                    v[P_INM2] += w == 2 ? mm : 0.0;
                    v[P_INM3] += w == 3 ? mm : 0.0;
                }
            }
        }
        if (!raw && wall) reconstruct_wall(c, x, qf, qg, qh);
        Macro<R> m;
        macros(c, qf, qg, qh, m);
        const int64_t o = kk;
        fields[0 * nn + o] = (double)m.ux;
        fields[1 * nn + o] = (double)m.uy;
        fields[2 * nn + o] = (double)m.Tf;
        fields[3 * nn + o] = (double)m.Tm;
        fields[4 * nn + o] = (double)m.fl;
        fields[5 * nn + o] = (double)m.rho;
        if (!finite) v[P_NF] = 1.0;
        if (!wall) {
            v[P_FL] = (double)m.fl;
            // phi rho_l H + (1-phi) rho_m c_pm T_m and rho, from the offsets
            double sg = 0.0, sh = 0.0, sf = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                sg += c.g_ref[i] + (double)qg[i];
                sh += c.h_ref[i] + (double)qh[i];
                sf += (double)w_of<double>(i) + (double)qf[i];
            }
            v[P_E] = c.we * sg + c.wm * sh;
            v[P_M] = sf;
            v[P_DT] = fabs((double)m.Tf - (double)m.Tm);
            v[P_U] = sqrt((double)m.ux * (double)m.ux + (double)m.uy * (double)m.uy);
        }
    }
    // Fixed-order tree reduction (deterministic).
    __shared__ double red[NPART][MB];
#pragma unroll
    for (int k = 0; k < NPART; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int st = MB / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
#pragma unroll
            for (int k = 0; k < NPART; ++k) {
                const double a = red[k][threadIdx.x], b = red[k][threadIdx.x + st];
                red[k][threadIdx.x] = (k == P_DT || k == P_U) ? fmax(a, b) : a + b;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < NPART) partials[(int64_t)blockIdx.x * NPART + threadIdx.x] = red[threadIdx.x][0];
}

template <typename S>
static hipError_t launch_macro_s(const MacroLaunch &L, int nx, int ny, hipStream_t s) {
    using R = typename RealOf<S>::type;
    hipLaunchKernelGGL((macro_kernel<S, R>), dim3(L.nblocks), dim3(MB), 0, s, (const S *)L.src,
                       L.plane_stride, (const CavityConst<R> *)L.cav, L.cav_index, L.raw, L.fields,
                       L.partials);
    return hipGetLastError();
}

hipError_t launch_macro(const MacroLaunch &L, int nx, int ny, hipStream_t s) {
    if (L.nblocks != macro_blocks(nx, ny)) return hipErrorInvalidValue;
    switch (L.storage) {
        case ST_F64: return launch_macro_s<double>(L, nx, ny, s);
        case ST_F32: return launch_macro_s<float>(L, nx, ny, s);
        case ST_F16: return launch_macro_s<__half>(L, nx, ny, s);
        case ST_BF16: return launch_macro_s<__hip_bfloat16>(L, nx, ny, s);
        default: return hipErrorInvalidValue;
    }
}

// Final pass: fixed-order sums of the block partials, Nusselt numbers from
// one-sided second-order differences, the melt front on the middle row and
// the wall tallies.
__global__ __launch_bounds__(MB) void diag_kernel(DiagLaunch L) {
    const int t = threadIdx.x;
    const int nx = L.nx, ny = L.ny;
    const int64_t nn = (int64_t)nx * ny;
    __shared__ double red[NPART + 3 + 8][MB];
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
    const double *Tf = L.fields + 2 * nn;
    const double *Tm = L.fields + 3 * nn;
    if (!L.periodic) {
        for (int y = 1 + t; y <= ny - 2; y += MB) {
            const int64_t r = (int64_t)y * nx;
            const double dTf = (-3.0 * Tf[r] + 4.0 * Tf[r + 1] - Tf[r + 2]) * 0.5;
            const double dTm = (-3.0 * Tm[r] + 4.0 * Tm[r + 1] - Tm[r + 2]) * 0.5;
            v[NPART + 0] += dTf;  // PCM-only gradient
            const double cTf = (3.0 * Tf[r + nx - 1] - 4.0 * Tf[r + nx - 2] + Tf[r + nx - 3]) * 0.5;
            const double cTm = (3.0 * Tm[r + nx - 1] - 4.0 * Tm[r + nx - 2] + Tm[r + nx - 3]) * 0.5;
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
#pragma unroll
    for (int k = 0; k < NPART + 11; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int st = MB / 2; st > 0; st >>= 1) {
        if (t < st) {
#pragma unroll
            for (int k = 0; k < NPART + 11; ++k) {
                const double a = red[k][t], b = red[k][t + st];
                red[k][t] = (k == P_DT || k == P_U) ? fmax(a, b) : a + b;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        double *o = L.out;
        const double nint = L.periodic ? (double)nx * (ny - 2) : (double)(nx - 2) * (ny - 2);
        o[D_FL] = red[P_FL][0] / nint;
        o[D_E] = red[P_E][0];
        o[D_M] = red[P_M][0];
        o[D_DT] = red[P_DT][0];
        o[D_U] = red[P_U][0];
        o[D_NF] = red[P_NF][0];
        const double nrow = (double)(ny - 2);
        o[D_NUH] = L.periodic ? 0.0 : -(L.L / (L.ke * L.dT)) * (red[NPART + 1][0] / nrow);
        o[D_NUHP] = L.periodic ? 0.0 : -(L.L / L.dT) * (red[NPART + 0][0] / nrow);
        o[D_NUC] = L.periodic ? 0.0 : -(L.L / (L.ke * L.dT)) * (red[NPART + 2][0] / nrow);
        // melt front: first f_l = 0.5 crossing on row ny/2 seen from x = 0
        double xf = 1.0;
        if (!L.periodic) {
            const double *fl = L.fields + 4 * nn + (int64_t)(ny / 2) * nx;
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
            o[D_FLUXE + w] = red[NPART + 3 + w][0] + red[P_INE0 + w][0];
            o[D_FLUXM + w] = red[NPART + 7 + w][0] + red[P_INM0 + w][0];
        }
    }
}

hipError_t launch_diag(const DiagLaunch &L, int nx, int ny, hipStream_t s) {
    if (L.nx != nx || L.ny != ny) return hipErrorInvalidValue;
    hipLaunchKernelGGL(diag_kernel, dim3(1), dim3(MB), 0, s, L);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Initial state: equilibria at rest (Eqs. 27, 40, 49) at the given
// temperatures, stored as offsets; the previous-step source equals the
// current one.
// ---------------------------------------------------------------------------
template <typename S, typename R>
__global__ __launch_bounds__(MB) void init_kernel(const CavityConst<R> *__restrict__ cav, int ci,
                                                  S *__restrict__ dst, int64_t stride,
                                                  R *__restrict__ sr,
                                                  const double *__restrict__ T_pcm,
                                                  const double *__restrict__ T_mf) {
    using C = Codec<S>;
    const CavityConst<R> &c = cav[ci];
    const int nx = c.nx, ny = c.ny;
    const int64_t nn = (int64_t)nx * ny;
    const int64_t kk = (int64_t)blockIdx.x * MB + threadIdx.x;
    if (kk >= nn) return;
    const int x = (int)(kk % nx);
    double Tf = T_pcm ? T_pcm[kk] : c.T_init;
    double Tm = T_mf ? T_mf[kk] : c.T_init;
    if (!c.periodic && x == 0) Tf = Tm = (double)c.T_hot;
    if (!c.periodic && x == nx - 1) Tf = Tm = (double)c.T_cold;
    // inverse of Eq. (38) (a tie at the solidus goes to the solid branch)
    const double Tfs = c.T_fs, Tfl = c.T_fl, Hfs = c.H_fs, Hfl = c.H_fl;
    double H;
    if (Tf <= Tfs) H = Tf / (double)c.inv_cps;
    else if (Tf >= Tfl) H = (Tf - Tfl) / (double)c.inv_cpl + Hfl;
    else H = Hfs + (Tf - Tfs) / (Tfl - Tfs) * (Hfl - Hfs);
    const double dT = Tf - (double)c.T_ref, dTm = Tm - (double)c.T_ref;
    const double dH = H - (double)c.H_ref;
    const double cf = c.c_fref, cm = c.c_mref, cpm = c.c_pm;
    const int64_t k = c.node0 + kk;
    for (int i = 0; i < 9; ++i) {
        const double wi = w_of<double>(i);
        const double qg = i == 0 ? dH - 5.0 / 9.0 * cf * dT : wi * cf * dT;
        const double qh = i == 0 ? (cpm - 5.0 / 9.0 * cm) * dTm : wi * cm * dTm;
        dst[(int64_t)i * stride + k] = C::from_double(0.0);
        dst[(int64_t)(9 + i) * stride + k] = C::from_double(qg * (double)c.scale[1]);
        dst[(int64_t)(18 + i) * stride + k] = C::from_double(qh * (double)c.scale[2]);
    }
    sr[k] = (R)((double)c.hv_f * (Tm - Tf));
}

template <typename S>
static hipError_t launch_init_s(const InitLaunch &L, int nx, int ny, hipStream_t s) {
    using R = typename RealOf<S>::type;
    const int nb = macro_blocks(nx, ny);
    hipLaunchKernelGGL((init_kernel<S, R>), dim3(nb), dim3(MB), 0, s, (const CavityConst<R> *)L.cav,
                       L.cav_index, (S *)L.dst, L.plane_stride, (R *)L.sr, L.T_pcm, L.T_mf);
    return hipGetLastError();
}

hipError_t launch_init(const InitLaunch &L, int nx, int ny, hipStream_t s) {
    switch (L.storage) {
        case ST_F64: return launch_init_s<double>(L, nx, ny, s);
        case ST_F32: return launch_init_s<float>(L, nx, ny, s);
        case ST_F16: return launch_init_s<__half>(L, nx, ny, s);
        case ST_BF16: return launch_init_s<__hip_bfloat16>(L, nx, ny, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename S>
__global__ void poke_kernel(S *p, double v) {
    *p = Codec<S>::from_double(v);
}

hipError_t launch_poke(int storage, void *ptr, double value, hipStream_t s) {
    switch (storage) {
        case ST_F64: hipLaunchKernelGGL(poke_kernel<double>, dim3(1), dim3(1), 0, s, (double *)ptr, value); break;
        case ST_F32: hipLaunchKernelGGL(poke_kernel<float>, dim3(1), dim3(1), 0, s, (float *)ptr, value); break;
        case ST_F16: hipLaunchKernelGGL(poke_kernel<__half>, dim3(1), dim3(1), 0, s, (__half *)ptr, value); break;
        case ST_BF16:
            hipLaunchKernelGGL(poke_kernel<__hip_bfloat16>, dim3(1), dim3(1), 0, s, (__hip_bfloat16 *)ptr, value);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
