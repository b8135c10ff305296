// Per-node arithmetic of the enthalpy-based MRT lattice Boltzmann method for
// solid-liquid phase change in metal foams under local thermal
// non-equilibrium (Liu, He & Li, arXiv:1701.00702): macroscopic values,
// the three moment-space collisions, wall reconstruction, and the storage
// layouts of the populations.  Everything here is __host__ __device__ so the
// kernels in lbm_kernels.hip and a host build of the same arithmetic share it.
//
// Populations are handled as offsets q_i = X_i - X_ref,i from a fixed
// reference equilibrium at rest (flow: w_i rho_0; enthalpy/metal: the
// equilibria at the middle of the mushy band on D2Q9, at the initial
// temperature on D2Q5, where a node the heat has not reached yet then holds
// exact zeros).  The moment algebra is affine, so the update runs on the
// offsets; in FP32 this keeps the small momentum of the Darcy-scale flow
// out of the rounding of O(1) populations.
//
// The thermal fields run on D2Q9 (Sec. III B/C) or on the D2Q5 lattice of
// Appendix B (its five velocities are the first five of Eq. 11); a layout
// carries the number QT of thermal velocities.  Population arrays are sized
// nine throughout; D2Q5 leaves entries 5..8 of g and h unused.
//
// Two arithmetic types: R for the flow and metal fields, RH for the PCM
// enthalpy field (H, T_f, f_l and the g collision).  The rest enthalpy
// population carries H itself, O(1), so its rounding is what limits FP32;
// the mixed form keeps that one population and the enthalpy arithmetic in
// FP64 and everything else in FP32.
#pragma once

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <type_traits>

#include "lbm_internal.h"

#define LBM_HD __host__ __device__ __forceinline__

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

// Reciprocal and square root of the velocity solve and the force: correctly
// rounded in FP64; in FP32 the hardware instructions (about 1 ulp), a tenth
// of the instructions of the correctly rounded sequences.  The FP32 forms
// are held to 1e-4 of the FP64 oracle, far above that rounding.
template <typename R>
LBM_HD R rcp_of(R x) {
    return R(1) / x;
}
template <typename R>
LBM_HD R sqrt_of(R x) {
    return sqrt(x);
}
#if defined(__HIP_DEVICE_COMPILE__)
template <>
LBM_HD float rcp_of<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}
template <>
LBM_HD float sqrt_of<float>(float x) {
    return __builtin_amdgcn_sqrtf(x);
}
#endif

// Fused multiply-add, rounded once.  The library is built without automatic
// contraction, so each fusion is written out here and every instantiation
// of the update rounds the same way.  With a power-of-two factor the fused
// form gives the same bits as the separate product and sum.
template <typename R>
LBM_HD R fma_of(R a, R b, R c) {
    return fma(a, b, c);
}
template <>
LBM_HD float fma_of<float>(float a, float b, float c) {
    return fmaf(a, b, c);
}

// Enthalpy-field constants in the enthalpy arithmetic type.
template <typename RH>
struct ThermalPick;
template <>
struct ThermalPick<float> {
    template <typename R>
    LBM_HD static const ThermalConst<float> &get(const CavityConst<R> &c) { return c.tf; }
};
template <>
struct ThermalPick<double> {
    template <typename R>
    LBM_HD static const ThermalConst<double> &get(const CavityConst<R> &c) { return c.td; }
};
template <typename RH, typename R>
LBM_HD const ThermalConst<RH> &thermal(const CavityConst<R> &c) {
    return ThermalPick<RH>::get(c);
}

// ---------------------------------------------------------------------------
// Streaming loads/stores and element codecs.  Every population is read and
// written once per step; whether the GPU accesses carry the non-temporal
// hint is a build option (LBM_NT_LOADS, LBM_NT_STORES).
// ---------------------------------------------------------------------------
#ifndef LBM_NT_LOADS
#define LBM_NT_LOADS 0
#endif
#ifndef LBM_NT_STORES
#define LBM_NT_STORES 1
#endif
template <typename T>
LBM_HD T ld_stream(const T *p) {
#if defined(__HIP_DEVICE_COMPILE__) && LBM_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
template <typename T>
LBM_HD void st_stream(T *p, T v) {
#if defined(__HIP_DEVICE_COMPILE__) && LBM_NT_STORES
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// A node's place in a population plane of a band block (the banded layout
// of the state buffers is described with CavityConst).  NodeRef: the node's
// offset rel within its band's plane plus the byte distance jump of its
// band's block from the block the plane pointer points into, both 32-bit;
// the step kernels use it with the same block for the whole workgroup (the
// tile's first band), so the address of each plane stays in scalar
// registers (the empty asm keeps the compiler from regrouping the sum into
// a per-lane 64-bit base plus plane offsets) and an access is that scalar
// base plus one 32-bit vector offset.  FarRef: the same in 64 bits, for an
// access anywhere in a cavity from its first band's block.
struct NodeRef {
    uint32_t rel, jump;
};
struct FarRef {
    int64_t rel, jump;
};
template <typename T>
using ByteOf = typename std::conditional<std::is_const<T>::value, const char, char>::type;
template <typename T>
LBM_HD T *at(T *plane, FarRef r) {
    return (T *)((ByteOf<T> *)(plane + r.rel) + r.jump);
}
template <typename T>
LBM_HD T *at(T *plane, NodeRef r) {
#if defined(__HIP_DEVICE_COMPILE__)
    __attribute__((address_space(1))) T *gp = (__attribute__((address_space(1))) T *)plane;  // global memory
    asm("" : "+s"(gp));
    plane = (T *)gp;
#endif
    return (T *)((ByteOf<T> *)plane + (r.rel * (uint32_t)sizeof(T) + r.jump));
}
// The address of a store of v to plane p (of stride elements) from base:
// as at(), with the plane's scalar base formed from a copy of the stride
// that depends on v.  The bases are then computed next to the stores, not
// shared with the loads' and held in scalar registers across the update.
template <typename T, typename V>
LBM_HD T *at_store(T *base, int p, int64_t stride, FarRef r, V v) {
    (void)v;
    return at(base + (int64_t)p * stride, r);
}
template <typename T, typename V>
LBM_HD T *at_store(T *base, int p, int64_t stride, NodeRef r, V v) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm("" : "+s"(stride) : "v"(v));
#else
    (void)v;
#endif
    return at(base + (int64_t)p * stride, r);
}

struct E64 {
    using T = double;
    LBM_HD static double dec(double v) { return v; }
    LBM_HD static double enc(double v) { return v; }
};
struct E32 {
    using T = float;
    LBM_HD static float dec(float v) { return v; }
    LBM_HD static float enc(float v) { return v; }
};
struct E16 {  // IEEE binary16, round to nearest even
    using T = uint16_t;
    LBM_HD static float dec(uint16_t v) { return (float)__builtin_bit_cast(_Float16, v); }
    LBM_HD static uint16_t enc(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
};
struct EB16 {  // bfloat16, round to nearest even (finite values)
    using T = uint16_t;
    LBM_HD static float dec(uint16_t v) { return __builtin_bit_cast(float, ((uint32_t)v) << 16); }
    LBM_HD static uint16_t enc(float v) {
        uint32_t u = __builtin_bit_cast(uint32_t, v);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    }
};

// ---------------------------------------------------------------------------
// Storage layouts.  load<V>() returns the offset q_i of field f (0 flow,
// 1 enthalpy, 2 metal), direction i, at packed node k, in type V; store()
// writes the offsets of one field at node k (nine for the flow, QT for the
// thermal fields).  beta is the per-node base value the split layout stores
// (unused elsewhere).
// ---------------------------------------------------------------------------

// 9 + 2 QT planes of one element type, [f0..f8, g0..g(QT-1), h0..h(QT-1)];
// 16-bit forms carry a power-of-two scale.
template <class E, bool SCALED, int QT_ = 9>
struct Plain {
    using T = typename E::T;
    using C = decltype(E::dec(T()));  // element arithmetic type of the codec
    static constexpr int QT = QT_;
    static constexpr int bytes_per_node = (9 + 2 * QT) * (int)sizeof(T);
    LBM_HD static int plane(int f, int i) { return f == 0 ? i : 9 + (f - 1) * QT + i; }
    template <typename V, typename R, typename K>
    LBM_HD static V load(const void *base, int64_t stride, int f, int i, K k, const CavityConst<R> &c) {
        const T *p = at((const T *)base + (int64_t)plane(f, i) * stride, k);
        const V v = (V)E::dec(ld_stream(p));
        return SCALED ? v * (V)c.inv_scale[f] : v;
    }
    template <typename V, typename R, typename K>
    LBM_HD static void store(void *base, int64_t stride, int f, const V q[9], V beta, K k,
                             const CavityConst<R> &c) {
        (void)beta;
        const int n = f == 0 ? 9 : QT;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (i < n) {
                const T e = E::enc((C)(SCALED ? q[i] * (V)c.scale[f] : q[i]));
                st_stream(at_store((T *)base, plane(f, i), stride, k, e), e);
            }
    }
};

// FP32 planes for all populations but the rest enthalpy one, which gets an
// FP64 plane: [f0..f8, g1..g(QT-1), h0..h(QT-1)] in FP32 (8 + 2 QT planes),
// then g0 in FP64; 112 bytes per node on D2Q9, 80 on D2Q5.
template <int QT_ = 9>
struct PlainH64 {
    static constexpr int QT = QT_;
    static constexpr int NF32 = 8 + 2 * QT;
    static constexpr int bytes_per_node = NF32 * 4 + 8;
    LBM_HD static int plane(int f, int i) { return f == 0 ? i : (f == 1 ? 8 + i : 8 + QT + i); }
    template <typename V, typename R, typename K>
    LBM_HD static V load(const void *base, int64_t stride, int f, int i, K k, const CavityConst<R> &c) {
        (void)c;
        if (f == 1 && i == 0) return (V)ld_stream(at((const double *)((const float *)base + NF32 * stride), k));
        return (V)ld_stream(at((const float *)base + (int64_t)plane(f, i) * stride, k));
    }
    template <typename V, typename R, typename K>
    LBM_HD static void store(void *base, int64_t stride, int f, const V q[9], V beta, K k,
                             const CavityConst<R> &c) {
        (void)beta;
        (void)c;
        const int n = f == 0 ? 9 : QT;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if (i >= n) continue;
            if (f == 1 && i == 0) {
                const double e = (double)q[0];
                st_stream(at_store((double *)((float *)base + NF32 * stride), 0, stride, k, e), e);
            } else {
                const float e = (float)q[i];
                st_stream(at_store((float *)base, plane(f, i), stride, k, e), e);
            }
        }
    }
};

// Split 16-bit layout: per field, the rest population and a base value beta
// in FP32, and the eight moving populations as 16-bit remainders (binary16,
// ER = E16, or bfloat16, ER = EB16) from the rest equilibrium of the base,
// r_i = q_i - w_i beta (scaled).  Bases: flow delta rho, enthalpy
// c_f,ref (T_f - T_ref), metal c_m,ref (T_m - T_ref); the moving populations
// stay close to w_i beta, so their remainders are small and 16 bits keep
// them to ~1e-3 (binary16) or ~8e-3 (bfloat16) relative, while the
// conserved content (rest population, base) keeps FP32 precision.
// Planes: 6 FP32 planes [q_f0, b_f, q_g0, b_g, q_h0, b_h] with b = w_1 beta
// (the axis weight 1/9 times the base), then 24 16-bit planes
// [field][direction 1..8]; 72 bytes per node.
// The split codec's arithmetic, shared by the global layout and its LDS
// copy: a population is w_i beta + r / s (r the 16-bit remainder, s the
// field's power-of-two scale).  With w_i beta = c_i b, c_i = 1 on the axes
// and 1/4 on the diagonals (exact), an axis population decodes with one
// fused multiply-add and a diagonal one with two operations, and a field's
// eight remainders q s - (c_i s) b take one fused multiply-add each after
// two products per field.  Rounding b once and scaling it by powers of two
// gives the same bits as rounding w_i beta per direction.
template <typename V>
__host__ __device__ constexpr V split_c(int i) {
    return i <= 4 ? V(1) : V(0.25);
}
template <typename V>
LBM_HD V split_base(V beta) {
    return w_of<V>(1) * beta;
}
template <typename V>
LBM_HD V split_dec(int i, V b, V r, V inv_scale) {
    return fma_of(r, inv_scale, split_c<V>(i) * b);
}
template <typename V>
LBM_HD float split_rem(int i, V q, V b, V scale) {
    return (float)fma_of(q, scale, -(split_c<V>(i) * scale) * b);
}

template <class ER>
struct SplitT {
    static constexpr int QT = 9;
    static constexpr int bytes_per_node = 6 * 4 + 24 * 2;
    // the stored base b of field f at node k
    template <typename K>
    LBM_HD static float load_base(const void *base, int64_t stride, int f, K k) {
        return ld_stream(at((const float *)base + (int64_t)(2 * f + 1) * stride, k));
    }
    // moving population i (>= 1) of field f at node k, given that node's base
    template <typename V, typename R, typename K>
    LBM_HD static V load_moving(const void *base, int64_t stride, int f, int i, K k, V b, const CavityConst<R> &c) {
        const uint16_t *Qp = (const uint16_t *)((const float *)base + 6 * stride);
        const V r = (V)ER::dec(ld_stream(at(Qp + (int64_t)(8 * f + i - 1) * stride, k)));
        return split_dec<V>(i, b, r, (V)c.inv_scale[f]);
    }
    template <typename V, typename R, typename K>
    LBM_HD static V load(const void *base, int64_t stride, int f, int i, K k, const CavityConst<R> &c) {
        const float *P = (const float *)base;
        if (i == 0) return (V)ld_stream(at(P + (int64_t)(2 * f) * stride, k));
        return load_moving<V>(base, stride, f, i, k, (V)load_base(base, stride, f, k), c);
    }
    template <typename V, typename R, typename K>
    LBM_HD static void store(void *base, int64_t stride, int f, const V q[9], V beta, K k,
                             const CavityConst<R> &c) {
        float *P = (float *)base;
        const float e0 = (float)q[0], eb = (float)split_base<V>(beta);
        st_stream(at_store(P, 2 * f, stride, k, e0), e0);
        st_stream(at_store(P, 2 * f + 1, stride, k, eb), eb);
        uint16_t *Qp = (uint16_t *)(P + 6 * stride);
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const uint16_t e = ER::enc(split_rem<V>(i, q[i], (V)eb, (V)c.scale[f]));
            st_stream(at_store(Qp, 8 * f + i - 1, stride, k, e), e);
        }
    }
};
using Split16 = SplitT<E16>;
using SplitB16 = SplitT<EB16>;

// Layout and arithmetic types of each storage form.
template <int ST>
struct LayoutOf;
template <>
struct LayoutOf<ST_F64> {
    using L = Plain<E64, false>;
    using R = double;
    using RH = double;
};
template <>
struct LayoutOf<ST_F32> {
    using L = Plain<E32, false>;
    using R = float;
    using RH = float;
};
template <>
struct LayoutOf<ST_F16> {
    using L = Plain<E16, true>;
    using R = float;
    using RH = float;
};
template <>
struct LayoutOf<ST_BF16> {
    using L = Plain<EB16, true>;
    using R = float;
    using RH = float;
};
template <>
struct LayoutOf<ST_F16S> {
    using L = Split16;
    using R = float;
    using RH = float;
};
template <>
struct LayoutOf<ST_BF16S> {
    using L = SplitB16;
    using R = float;
    using RH = float;
};
template <>
struct LayoutOf<ST_F32H> {
    using L = PlainH64<9>;
    using R = float;
    using RH = double;
};
template <>
struct LayoutOf<ST5_F64> {
    using L = Plain<E64, false, 5>;
    using R = double;
    using RH = double;
};
template <>
struct LayoutOf<ST5_F32> {
    using L = Plain<E32, false, 5>;
    using R = float;
    using RH = float;
};
template <>
struct LayoutOf<ST5_F32H> {
    using L = PlainH64<5>;
    using R = float;
    using RH = double;
};

// ---------------------------------------------------------------------------
// Moment transforms of Eq. (13) on offsets.  d = M q, and q = M^-1 d with
// M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4): the
// inverse takes the scaled moments a_k = d_k / |M_k|^2 (|M_k|^2 the squared
// norm of row k of M), whose factors the collisions fold into their rates.
// ---------------------------------------------------------------------------
template <typename R>
LBM_HD void to_moments(const R q[9], R d[9]) {
    const R p13 = q[1] + q[3], p24 = q[2] + q[4], m13 = q[1] - q[3], m24 = q[2] - q[4];
    const R p56 = q[5] + q[6], p78 = q[7] + q[8], m56 = q[5] - q[6], m78 = q[7] - q[8];
    const R s14 = p13 + p24, s58 = p56 + p78;
    const R dxd = m56 - m78, dyd = p56 - p78;
    d[0] = (q[0] + s14) + s58;
    d[1] = fma_of(R(2), s58, fma_of(R(-4), q[0], -s14));
    d[2] = fma_of(R(4), q[0], fma_of(R(-2), s14, s58));
    d[3] = m13 + dxd;
    d[4] = fma_of(R(-2), m13, dxd);
    d[5] = m24 + dyd;
    d[6] = fma_of(R(-2), m24, dyd);
    d[7] = p13 - p24;
    d[8] = m56 + m78;
}

// 1 / |M_k|^2.
template <typename R>
__host__ __device__ constexpr R moment_norm(int k) {
    return k == 0 ? R(1) / R(9) : (k <= 2 ? R(1) / R(36) : (k == 3 || k == 5 ? R(1) / R(6) : (k <= 6 ? R(1) / R(12) : R(0.25))));
}

template <typename R>
LBM_HD void from_scaled(const R a[9], R q[9]) {
    const R axis = fma_of(R(-2), a[2], a[0] - a[1]);
    const R diag = fma_of(R(2), a[1], a[0]) + a[2];
    const R xa = fma_of(R(-2), a[4], a[3]), ya = fma_of(R(-2), a[6], a[5]);
    const R xd = a[3] + a[4], yd = a[5] + a[6];
    const R ap = axis + a[7], am = axis - a[7];
    const R dp = diag + a[8], dm = diag - a[8];
    const R u = xd + yd, v = xd - yd;
    q[0] = fma_of(R(4), a[2], fma_of(R(-4), a[1], a[0]));
    q[1] = ap + xa;
    q[3] = ap - xa;
    q[2] = am + ya;
    q[4] = am - ya;
    q[5] = dp + u;
    q[7] = dp - u;
    q[6] = dm - v;
    q[8] = dm + v;
}

// D2Q5 transforms of Eq. (B1) on offsets: d = M q, and its inverse
// q0 = d0 - d3, q1,3 = (d3 + d4)/4 +- d1/2, q2,4 = (d3 - d4)/4 +- d2/2,
// taken from e_k = g_k d_k with g = (1, 1/2, 1/2, 1/4, 1/4), whose factors
// the collisions fold into their rates (powers of two: the same bits).
template <typename R>
LBM_HD void to_moments5(const R q[9], R d[5]) {
    const R ax = q[1] + q[3], ay = q[2] + q[4];
    d[0] = ((q[0] + q[1]) + (q[2] + q[3])) + q[4];
    d[1] = q[1] - q[3];
    d[2] = q[2] - q[4];
    d[3] = ax + ay;
    d[4] = ax - ay;
}

template <typename R>
LBM_HD void from_scaled5(const R e[5], R q[9]) {
    const R a = e[3] + e[4], b = e[3] - e[4];
    q[0] = fma_of(R(-4), e[3], e[0]);
    q[1] = a + e[1];
    q[3] = a - e[1];
    q[2] = b + e[2];
    q[4] = b - e[2];
}

// ---------------------------------------------------------------------------
// Macroscopic values of one node from its post-streaming offsets.
// ---------------------------------------------------------------------------
template <typename RH>
struct Thermo {  // PCM enthalpy field, Eqs. (37)-(39)
    RH dH, H, Tf, fl;
};
template <typename R>
struct Macro {  // everything the flow and metal collisions need
    R Tf, fl, dTm, Tm, drho, rho, ux, uy, umag, Gx, Gy;
};

// Eqs. (38)-(39), branches in the order the paper lists them.
template <typename RH>
LBM_HD void eos(const ThermalConst<RH> &t, RH H, RH &T, RH &fl) {
    if (H <= t.H_fs) {
        T = H * t.inv_cps;
        fl = RH(0);
    } else if (H >= t.H_fl) {
        T = t.T_fl + (H - t.H_fl) * t.inv_cpl;
        fl = RH(1);
    } else {
        fl = (H - t.H_fs) * t.inv_dH;
        T = t.T_fs + fl * t.dT_band;
    }
}

// Moments of the three fields' post-streaming offsets, Eq. (13) (D2Q5
// thermal fields: Eq. B1).  Their zeroth moments are delta rho, delta H
// (Eq. 37) and c_pm delta T_m (Eq. 48).
//
// Split enthalpy arithmetic (RH wider than R, the form with the FP64 rest
// enthalpy population): the rest population q_0 carries H, O(1), while the
// moving ones are small.  The moments g are then taken in R of the moving
// populations alone (q_0 read as zero) and q_0 is kept in RH as `rest`.
// Column 0 of the transform is (1, -4, 4, 0, ..., 0) (D2Q5: (1, 0, ..., 0)),
// and the enthalpy equilibrium moves with H along the same column (Eq. 34:
// n_1^eq = -4 H + ..., n_2^eq = 4 H - ...; Eq. B2: only n_0^eq), so the
// collision of the moving part yields every post-collision population, and
// the rest one is q_0 plus the moving part's rest result: q_0 enters no
// rounding but that of one addition in RH.
template <typename R, typename RH>
struct Moments {
    static constexpr bool SPLIT = !std::is_same<R, RH>::value;
    using RG = typename std::conditional<SPLIT, R, RH>::type;
    R f[9], h[9];
    RG g[9];
    RH rest;  // SPLIT: the rest enthalpy population q_0
};
template <int QT, typename R, typename RH>
LBM_HD void field_moments(const R qf[9], const RH qg[9], const R qh[9], Moments<R, RH> &mo) {
    using Mo = Moments<R, RH>;
    using RG = typename Mo::RG;
    to_moments(qf, mo.f);
    RG qs[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) qs[i] = Mo::SPLIT && i == 0 ? RG(0) : (RG)qg[i];
    mo.rest = Mo::SPLIT ? qg[0] : RH(0);
    if (QT == 9) {
        to_moments(qs, mo.g);
        to_moments(qh, mo.h);
    } else {
        to_moments5(qs, mo.g);
        to_moments5(qh, mo.h);
    }
}

// Everything the collisions need, from the moments; blends the flow moments
// in place (Eq. 20: f = f_l f+ + (1 - f_l) w rho, whose moments on offsets
// are f_l d + (1 - f_l) delta rho (1, -2, 1, 0, ..., 0), M w having the
// moments (1, -2, 1, 0, ..., 0)).  The bounce-back alternative of Sec. V B
// keeps f+ unblended.
template <int QT, typename R, typename RH>
LBM_HD void macros_of(const CavityConst<R> &c, Moments<R, RH> &mo, Thermo<RH> &th, Macro<R> &m) {
    const ThermalConst<RH> &t = thermal<RH>(c);
    // Eq. (37), Eqs. (38)-(39)
    th.dH = Moments<R, RH>::SPLIT ? (RH)mo.g[0] + mo.rest : (RH)mo.g[0];
    th.H = t.H_ref + th.dH;
    eos(t, th.H, th.Tf, th.fl);
    m.Tf = (R)th.Tf;
    m.fl = (R)th.fl;
    // Eq. (48)
    m.dTm = mo.h[0] * c.inv_cpm;
    m.Tm = c.T_ref + m.dTm;
    // Eq. (21)
    m.drho = mo.f[0];
    m.rho = R(1) + m.drho;
    if (!c.bounce_back) {
        const R sol = (R(1) - m.fl) * m.drho;
        mo.f[0] = m.drho;
        mo.f[1] = fma_of(m.fl, mo.f[1], R(-2) * sol);
        mo.f[2] = fma_of(m.fl, mo.f[2], sol);
#pragma unroll
        for (int k = 3; k < 9; ++k) mo.f[k] = m.fl * mo.f[k];
    }
    // Eq. (7): buoyancy along +axis (gravity along -axis).
    const R G = c.gbeta * (m.Tf - c.T0) * m.fl;
    m.Gx = c.gaxis == 0 ? G : R(0);
    m.Gy = c.gaxis == 1 ? G : R(0);
    // Eq. (24) (j = the blended moments 3 and 5), then the explicit root
    // Eq. (23) with Eq. (25).
    const R jx = mo.f[3], jy = mo.f[5];
    const R inv_rho = rcp_of(m.rho);
    const R vx = fma_of(jx, inv_rho, R(0.5) * c.phi * m.Gx);
    const R vy = fma_of(jy, inv_rho, R(0.5) * c.phi * m.Gy);
    const R vmag = sqrt_of(fma_of(vx, vx, vy * vy));
    const R inv_den = rcp_of(c.l0 + sqrt_of(fma_of(c.l1, vmag, c.l0sq)));
    m.ux = vx * inv_den;
    m.uy = vy * inv_den;
    m.umag = vmag * inv_den;  // |u| of Eq. (3)
    // bounce-back: below the interface value f_l = 0.5 a node is solid, at rest
    if (c.bounce_back && m.fl < R(0.5)) {
        m.ux = R(0);
        m.uy = R(0);
        m.umag = R(0);
    }
}

// The same from populations (wall partners, diagnostics).
template <int QT, typename R, typename RH>
LBM_HD void macros(const CavityConst<R> &c, const R qf[9], const RH qg[9], const R qh[9], Thermo<RH> &th,
                   Macro<R> &m) {
    Moments<R, RH> mo;
    field_moments<QT>(qf, qg, qh, mo);
    macros_of<QT>(c, mo, th, m);
}

// Flow collision, Eqs. (14), (16)-(19), from the blended moments d (into q);
// with the bounce-back alternative (Sec. V B) a solid node instead returns
// every population of q along the opposite link (the reference w_i rho_0 is
// symmetric, so the offsets swap the same way).
template <typename R>
LBM_HD void collide_flow(const CavityConst<R> &c, const Macro<R> &m, R d[9], R q[9]) {
    if (c.bounce_back && m.fl < R(0.5)) {
        R t;
        t = q[1]; q[1] = q[3]; q[3] = t;
        t = q[2]; q[2] = q[4]; q[4] = t;
        t = q[5]; q[5] = q[7]; q[7] = t;
        t = q[6]; q[6] = q[8]; q[8] = t;
        return;
    }
    const R ux = m.ux, uy = m.uy, rho = m.rho;
    const R uu = fma_of(ux, ux, uy * uy);
    // Eq. (3): F = -(drag_lin + drag_quad |u|) u + phi G
    const R drag = fma_of(c.drag_quad, m.umag, c.drag_lin);
    const R Fx = fma_of(-drag, ux, c.phi * m.Gx);
    const R Fy = fma_of(-drag, uy, c.phi * m.Gy);
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
    // scaled post-collision moments: ((1 - s) d + s eq + (1 - s/2) S) / |M_k|^2
    R a[9];
    a[0] = m.drho * moment_norm<R>(0);
#pragma unroll
    for (int k = 1; k < 9; ++k) a[k] = fma_of(c.fC[k], S[k], fma_of(c.fB[k], eq[k], c.fA[k] * d[k]));
    from_scaled(a, q);
}

// Post-collision enthalpy offsets from the collision's output qs (in the
// moment type RG): the rest population adds q_0 back in the split form.
template <typename RG, typename RH>
LBM_HD void pcm_out(const RG qs[9], RH rest, RH q[9]) {
    constexpr bool SPLIT = !std::is_same<RG, RH>::value;
#pragma unroll
    for (int i = 0; i < 9; ++i) q[i] = SPLIT && i == 0 ? rest + (RH)qs[0] : (RH)qs[i];
}

// PCM enthalpy collision, Eqs. (32), (34)-(35), from the moments d (in RG,
// of the moving populations alone in the split form, where rest is q_0; d_0
// is then delta H - q_0, and the equilibrium of Eq. 34 is taken at it).
template <typename R, typename RH, typename RG>
LBM_HD void collide_pcm(const CavityConst<R> &c, const Thermo<RH> &th, const Macro<R> &m, RH S_pcm,
                        RG d[9], RH rest, RH q[9]) {
    const ThermalConst<RG> &t = thermal<RG>(c);
    const RG dT = (RG)(th.Tf - thermal<RH>(c).T_ref);
    const RG jT = t.c_pl * (RG)th.Tf * t.inv_phi;
    const RG S = (RG)S_pcm;
    RG eq[7];  // eq_0 = d_0; eq_7 = eq_8 = 0
    eq[1] = -RG(4) * d[0] + RG(2) * t.c_fref * dT;
    eq[2] = RG(4) * d[0] - RG(3) * t.c_fref * dT;
    eq[3] = jT * (RG)m.ux;
    eq[4] = -eq[3];
    eq[5] = jT * (RG)m.uy;
    eq[6] = -eq[5];
    // scaled moments ((1 - zeta) d + zeta eq + S (1, -2, 1, 0, ...)) / |M_k|^2;
    // the zeroth moment is conserved (d_0 = eq_0), only S moves it
    RG a[9];
    a[0] = (d[0] + S) * moment_norm<RG>(0);
    a[1] = fma_of(RG(-2) * moment_norm<RG>(1), S, fma_of(t.zB[1], eq[1], t.zA[1] * d[1]));
    a[2] = fma_of(moment_norm<RG>(2), S, fma_of(t.zB[2], eq[2], t.zA[2] * d[2]));
#pragma unroll
    for (int k = 3; k < 7; ++k) a[k] = fma_of(t.zB[k], eq[k], t.zA[k] * d[k]);
    a[7] = t.zA[7] * d[7];
    a[8] = t.zA[8] * d[8];
    RG qs[9];
    from_scaled(a, qs);
    pcm_out(qs, rest, q);
}

// Metal-foam collision, Eqs. (43), (45)-(46).
template <typename R>
LBM_HD void collide_metal(const CavityConst<R> &c, const Macro<R> &m, R S_metal, R d[9], R q[9]) {
    R eq[3];  // eq_3 .. eq_8 = 0
    eq[0] = c.c_pm * m.dTm;
    eq[1] = (-R(4) * c.c_pm + R(2) * c.c_mref) * m.dTm;
    eq[2] = (R(4) * c.c_pm - R(3) * c.c_mref) * m.dTm;
    // scaled moments ((1 - eta) d + eta eq + S (1, -2, 1, 0, ...)) / |M_k|^2
    R a[9];
    a[0] = fma_of(moment_norm<R>(0), S_metal, fma_of(c.mB[0], eq[0], c.mA[0] * d[0]));
    a[1] = fma_of(R(-2) * moment_norm<R>(1), S_metal, fma_of(c.mB[1], eq[1], c.mA[1] * d[1]));
    a[2] = fma_of(moment_norm<R>(2), S_metal, fma_of(c.mB[2], eq[2], c.mA[2] * d[2]));
#pragma unroll
    for (int k = 3; k < 9; ++k) a[k] = c.mA[k] * d[k];
    from_scaled(a, q);
}

// D2Q5 enthalpy collision (Appendix B): equilibrium moments Eq. (B2) on
// offsets, Theta in the moment order of Eq. (B1), source S (1, 0, 0, varpi, 0);
// scaled moments e_k = g_k ((1 - zeta_k) d_k + zeta_k eq_k + S_k), the
// zeroth moment conserved (d_0 = eq_0 = delta H) so only S moves it.
template <typename R, typename RH, typename RG>
LBM_HD void collide_pcm5(const CavityConst<R> &c, const Thermo<RH> &th, const Macro<R> &m, RH S_pcm,
                         RG d[9], RH rest, RH q[9]) {
    const ThermalConst<RG> &t = thermal<RG>(c);
    const RG jT = t.c_pl * (RG)th.Tf * t.inv_phi;
    const RG eq1 = jT * (RG)m.ux, eq2 = jT * (RG)m.uy;  // eq_4 = 0
    const RG eq3 = t.varpi * t.c_fref * (RG)(th.Tf - thermal<RH>(c).T_ref);
    const RG S = (RG)S_pcm;
    RG e[5];
    e[0] = d[0] + S;
    e[1] = fma_of(t.zB[1], eq1, t.zA[1] * d[1]);
    e[2] = fma_of(t.zB[2], eq2, t.zA[2] * d[2]);
    e[3] = fma_of(t.varpi * RG(0.25), S, fma_of(t.zB[3], eq3, t.zA[3] * d[3]));
    e[4] = t.zA[4] * d[4];
    RG qs[9];
    from_scaled5(e, qs);
    qs[5] = qs[6] = qs[7] = qs[8] = RG(0);
    pcm_out(qs, rest, q);
}

// D2Q5 metal-foam collision (Appendix B): Eq. (B4), Q, S (1, 0, 0, varpi, 0),
// in the scaled moments of from_scaled5.
template <typename R>
LBM_HD void collide_metal5(const CavityConst<R> &c, const Macro<R> &m, R S_metal, R d[9], R q[9]) {
    const R eq0 = c.c_pm * m.dTm, eq3 = c.varpi * c.c_mref * m.dTm;  // eq_1 = eq_2 = eq_4 = 0
    R e[5];
    e[0] = fma_of(c.mB[0], eq0, c.mA[0] * d[0]) + S_metal;
    e[1] = c.mA[1] * d[1];
    e[2] = c.mA[2] * d[2];
    e[3] = fma_of(c.varpi * R(0.25), S_metal, fma_of(c.mB[3], eq3, c.mA[3] * d[3]));
    e[4] = c.mA[4] * d[4];
    from_scaled5(e, q);
}

// Wall whose thermal condition a wall node carries: an isothermal vertical
// wall, else an isothermal horizontal wall, else -1 (adiabatic: the node
// copies its partner's temperature).
template <typename R>
LBM_HD int thermal_wall(const CavityConst<R> &c, int x, int y) {
    const int v = c.periodic ? -1 : (x == 0 ? W_LEFT : (x == c.nx - 1 ? W_RIGHT : -1));
    const int h = y == 0 ? W_BOTTOM : (y == c.ny - 1 ? W_TOP : -1);
    if (v >= 0 && c.wall_iso[v]) return v;
    if (h >= 0 && c.wall_iso[h]) return h;
    return -1;
}

// Non-equilibrium extrapolation for wall node (x, y), applied in place to
// the partner's pulled offsets (Eq. 52 with wall velocity 0; thermal
// analogues with the isothermal or zero-gradient wall values).
template <int QT, typename R, typename RH>
LBM_HD void reconstruct_wall(const CavityConst<R> &c, int x, int y, R qf[9], RH qg[9], R qh[9]) {
    const ThermalConst<RH> &t = thermal<RH>(c);
    Thermo<RH> pt;
    Macro<R> p;
    macros<QT>(c, qf, qg, qh, pt, p);
    RH Tb, Hb;
    R Tmb;
    const int w = thermal_wall(c, x, y);
    if (w >= 0) {
        Tb = t.T_wall[w];
        Hb = t.H_wall[w];
        Tmb = c.T_wall[w];
    } else {
        Tb = pt.Tf;
        Hb = pt.H;
        Tmb = p.Tm;
    }
    const R uu = p.ux * p.ux + p.uy * p.uy;
    const RH dTg = Tb - pt.Tf;
    const R dTh = Tmb - p.Tm;
    // g^eq(H_b, T_b, 0) - g^eq(H, T, u) from Eq. (40) / Eq. (B3); h likewise
    // from Eq. (49) / Eq. (B5)
    const RH jT = t.inv_cs2 * t.c_pl * pt.Tf * t.inv_phi;
    qf[0] += -w_of<R>(0) * p.rho * (-R(1.5) * uu * c.inv_phi);
    if (QT == 9) {
        qg[0] += (Hb - pt.H) - RH(5) / RH(9) * t.c_fref * dTg;
        qh[0] += (c.c_pm - R(5) / R(9) * c.c_mref) * dTh;
    } else {
        qg[0] += (Hb - pt.H) - t.varpi * t.c_fref * dTg;
        qh[0] += (c.c_pm - c.varpi * c.c_mref) * dTh;
    }
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const R eu = R(ex_of(i)) * p.ux + R(ey_of(i)) * p.uy;
        // f^eq(rho, 0) - f^eq(rho, u) from Eq. (27)
        qf[i] += -w_of<R>(i) * p.rho * (R(3) * eu + R(4.5) * eu * eu * c.inv_phi - R(1.5) * uu * c.inv_phi);
        if (i < QT) {
            const RH wg = QT == 9 ? w_of<RH>(i) : RH(0.25) * t.varpi;
            const R wh = QT == 9 ? w_of<R>(i) : R(0.25) * c.varpi;
            qg[i] += wg * (t.c_fref * dTg - jT * (RH)eu);
            qh[i] += wh * c.c_mref * dTh;
        }
    }
}

// Wall classification and the node whose populations a node pulls: its own
// neighbourhood, or its interior partner's for a wall node (inward normal
// neighbour, diagonal at corners).
struct NodeGeom {
    bool wall, near_x, near_y;
    int sx, sy;
};

template <typename R>
LBM_HD NodeGeom geometry(const CavityConst<R> &c, int x, int y, bool pull) {
    NodeGeom g;
    const int nx = c.nx, ny = c.ny;
    const bool vwall = !c.periodic && (x == 0 || x == nx - 1);
    const bool hwall = (y == 0 || y == ny - 1);
    g.wall = vwall || hwall;
    g.sx = x;
    g.sy = y;
    if (pull && g.wall) {
        if (!c.periodic) g.sx = (x == 0) ? 1 : ((x == nx - 1) ? nx - 2 : x);
        g.sy = (y == 0) ? 1 : ((y == ny - 1) ? ny - 2 : y);
    }
    g.near_x = !g.wall && !c.periodic && (x == 1 || x == nx - 2);
    g.near_y = !g.wall && (y == 1 || y == ny - 2);
    return g;
}

// Position of wall node r of the bottom and top rows (the wall columns are
// handled with their rows).
template <typename R>
LBM_HD void ring_node(const CavityConst<R> &c, int r, int &x, int &y) {
    const int nx = c.nx;
    if (r < nx) {
        x = r;
        y = 0;
    } else {
        x = r - nx;
        y = c.ny - 1;
    }
}

// Where node (x, y) of a cavity sits relative to a band block.  BandOrigin:
// rows of band ba and ba + 1 from band ba's block (the step kernels' tiles
// span at most two bands).  AnyBand: any row, from the cavity's first block.
struct BandOrigin {
    int y_first, y_next;  // first rows of bands ba and ba + 1
    int pitch;
    uint32_t band_bytes;
    LBM_HD NodeRef operator()(int x, int y) const {
        return y < y_next ? NodeRef{(uint32_t)((y - y_first) * pitch + x), 0u}
                          : NodeRef{(uint32_t)((y - y_next) * pitch + x), band_bytes};
    }
    // row y resolved to its band once; node x of it by at_row
    LBM_HD NodeRef row(int y) const { return (*this)(0, y); }
    LBM_HD static NodeRef at_row(NodeRef r, int x) { return NodeRef{r.rel + (uint32_t)x, r.jump}; }
};
struct AnyBand {
    int band_rows, pitch;
    int64_t band_bytes;
    LBM_HD FarRef operator()(int x, int y) const {
        const int b = y / band_rows;
        return FarRef{(int64_t)(y - b * band_rows) * pitch + x, (int64_t)b * band_bytes};
    }
    LBM_HD FarRef row(int y) const { return (*this)(0, y); }
    LBM_HD static FarRef at_row(FarRef r, int x) { return FarRef{r.rel + x, r.jump}; }
};
template <typename R>
LBM_HD BandOrigin band_origin(const CavityConst<R> &c, int y) {  // from the band of row y
    const int ba = y / c.band_rows;
    return BandOrigin{ba * c.band_rows, (ba + 1) * c.band_rows, c.pitch, (uint32_t)c.band_bytes};
}
template <typename R>
LBM_HD AnyBand any_band(const CavityConst<R> &c) {
    return AnyBand{c.band_rows, c.pitch, c.band_bytes};
}
// The block of band b of cavity c in a state buffer.
template <typename R, typename V>
LBM_HD V *band_block(const CavityConst<R> &c, V *buf, int b) {
    return (V *)((ByteOf<V> *)buf + c.pop_off + (int64_t)b * c.band_bytes);
}
// Index of node (x, y) in the flat per-node arrays (interstitial source).
template <typename R>
LBM_HD int64_t flat_index(const CavityConst<R> &c, int x, int y) {
    return c.node0 + (int64_t)y * c.nx + x;
}

// Offsets of the node's post-streaming populations: pulled from the
// neighbours (Eqs. 15, 33, 44), or read in place for the initial state.
// src is the band block addr is relative to.
template <class Lay, typename R, typename RH, bool PULL, class A>
LBM_HD void gather_at(const CavityConst<R> &c, const void *src, const NodeGeom &g, int x, int y, A addr,
                      R qf[9], RH qg[9], R qh[9]) {
    const int nx = c.nx;
    const int64_t stride = c.band_nodes;
    if (PULL && !c.periodic) {
        // no wrap: the three rows the pulls read are resolved to their bands
        // once, and each pull is an offset within its row
        const auto row_up = addr.row(g.sy + 1), row_mid = addr.row(g.sy), row_down = addr.row(g.sy - 1);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const auto k = A::at_row(ey_of(i) > 0 ? row_down : (ey_of(i) < 0 ? row_up : row_mid), g.sx - ex_of(i));
            qf[i] = Lay::template load<R>(src, stride, 0, i, k, c);
            if (i < Lay::QT) {
                qg[i] = Lay::template load<RH>(src, stride, 1, i, k, c);
                qh[i] = Lay::template load<R>(src, stride, 2, i, k, c);
            } else {
                qg[i] = RH(0);
                qh[i] = R(0);
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int px = x, py = y;
        if (PULL) {
            px = g.sx - ex_of(i);
            if (c.periodic) px = px < 0 ? px + nx : (px >= nx ? px - nx : px);
            py = g.sy - ey_of(i);
        }
        const auto k = addr(px, py);
        qf[i] = Lay::template load<R>(src, stride, 0, i, k, c);
        if (i < Lay::QT) {
            qg[i] = Lay::template load<RH>(src, stride, 1, i, k, c);
            qh[i] = Lay::template load<R>(src, stride, 2, i, k, c);
        } else {
            qg[i] = RH(0);
            qh[i] = R(0);
        }
    }
}

// From a whole state buffer.
template <class Lay, typename R, typename RH, bool PULL>
LBM_HD void gather(const CavityConst<R> &c, const void *buf, const NodeGeom &g, int x, int y, R qf[9],
                   RH qg[9], R qh[9]) {
    gather_at<Lay, R, RH, PULL>(c, band_block(c, buf, 0), g, x, y, any_band(c), qf, qg, qh);
}

// Energy and mass carried by direction i of the given offsets (FP64);
// energy moves only along the thermal lattice's links.
template <int QT, typename R, typename RH>
LBM_HD void link_content(const CavityConst<R> &c, int i, const R qf[9], const RH qg[9], const R qh[9],
                         double &e, double &m) {
    e = i < QT ? c.we * (c.g_ref[i] + (double)qg[i]) + c.wm * (c.h_ref[i] + (double)qh[i]) : 0.0;
    m = (double)w_of<double>(i) + (double)qf[i];
}

// The update of one node from its gathered (post-streaming) offsets: wall
// tallies (only when the node's step is counted here, `tally`), wall
// reconstruction, macroscopic values, the three collisions and the
// interstitial sources.  On return q* hold the post-collision offsets and
// m, th the values the split layout stores as bases; the result is the
// new PCM source Sr_f.
template <int QT, typename R, typename RH, bool PULL>
LBM_HD RH update_node(const CavityConst<R> &c, const NodeGeom &g, int x, int y, R qf[9], RH qg[9], R qh[9],
                      R sr_prev, bool tally, double *__restrict__ acc, Thermo<RH> &th, Macro<R> &m) {
    const int nx = c.nx, ny = c.ny;
    // Wall tallies: an interior node next to a wall owns one slot per wall it
    // touches (x: the vertical wall, y: the horizontal one).
    double xE = 0.0, xM = 0.0, yE = 0.0, yM = 0.0;
    if (PULL && tally && (g.near_x || g.near_y)) {
        // inflow: populations pulled from wall nodes (post-collision of the
        // previous step)
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int px = x - ex_of(i), py = y - ey_of(i);
            const bool onx = !c.periodic && (px == 0 || px == nx - 1);
            const bool ony = (py == 0 || py == ny - 1);
            if (onx || ony) {
                double e, mm;
                link_content<QT>(c, i, qf, qg, qh, e, mm);
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

    if (PULL && g.wall) reconstruct_wall<QT>(c, x, y, qf, qg, qh);

    Moments<R, RH> mo;
    field_moments<QT>(qf, qg, qh, mo);
    macros_of<QT>(c, mo, th, m);
    collide_flow(c, m, mo.f, qf);
    // Eqs. (36), (47) with the backward difference of Remark III.
    const RH srf = (RH)c.hv_f * ((RH)m.Tm - th.Tf);
    const R srm = c.hv_m * (m.Tf - m.Tm);
    const R srm_prev = -c.sr_ratio * sr_prev;
    const RH S_pcm = srf + RH(0.5) * (srf - (RH)sr_prev);
    const R S_metal = srm + R(0.5) * (srm - srm_prev);
    if (QT == 9) {
        collide_pcm(c, th, m, S_pcm, mo.g, mo.rest, qg);
        collide_metal(c, m, S_metal, mo.h, qh);
    } else {
        collide_pcm5(c, th, m, S_pcm, mo.g, mo.rest, qg);
        collide_metal5(c, m, S_metal, mo.h, qh);
    }

    if (tally && (g.near_x || g.near_y)) {
        // outflow: post-collision populations aimed at wall nodes
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int tx = x + ex_of(i), ty = y + ey_of(i);
            const bool onx = !c.periodic && (tx == 0 || tx == nx - 1);
            const bool ony = (ty == 0 || ty == ny - 1);
            if (onx || ony) {
                double e, mm;
                link_content<QT>(c, i, qf, qg, qh, e, mm);
                if (onx) {
                    xE -= e;
                    xM -= mm;
                } else {
                    yE -= e;
                    yM -= mm;
                }
            }
        }
        if (g.near_x) {
            const int64_t slot = c.acc0 + (x == 1 ? y : ny + y);
            acc[2 * slot] += xE;
            acc[2 * slot + 1] += xM;
        }
        if (g.near_y) {
            const int64_t slot = c.acc0 + 2 * ny + (y == 1 ? x : nx + x);
            acc[2 * slot] += yE;
            acc[2 * slot + 1] += yM;
        }
    }
    return srf;
}

// One node's full time step; addr places the node and its neighbours
// relative to the band blocks src and dst.
template <class Lay, typename R, typename RH, bool PULL, class A>
LBM_HD void step_node_at(const CavityConst<R> &c, const void *src, void *dst, const R *__restrict__ sr_src,
                         R *__restrict__ sr_dst, double *__restrict__ acc, int x, int y, A addr) {
    const NodeGeom g = geometry(c, x, y, PULL);
    R qf[9], qh[9];
    RH qg[9];
    gather_at<Lay, R, RH, PULL>(c, src, g, x, y, addr, qf, qg, qh);
    const auto k = addr(x, y);
    const int64_t kf = flat_index(c, x, y);
    Thermo<RH> th;
    Macro<R> m;
    const RH srf = update_node<Lay::QT, R, RH, PULL>(c, g, x, y, qf, qg, qh, sr_src[kf], true, acc, th, m);
    const ThermalConst<RH> &t = thermal<RH>(c);
    const int64_t stride = c.band_nodes;
    Lay::template store<R>(dst, stride, 0, qf, m.drho, k, c);
    Lay::template store<RH>(dst, stride, 1, qg, t.c_fref * (th.Tf - t.T_ref), k, c);
    Lay::template store<R>(dst, stride, 2, qh, c.c_mref * m.dTm, k, c);
    sr_dst[kf] = (R)srf;
}

// The same on whole state buffers.
template <class Lay, typename R, typename RH, bool PULL>
LBM_HD void step_node(const CavityConst<R> &c, const void *src, void *dst, const R *__restrict__ sr_src,
                      R *__restrict__ sr_dst, double *__restrict__ acc, int x, int y) {
    step_node_at<Lay, R, RH, PULL>(c, band_block(c, src, 0), band_block(c, dst, 0), sr_src, sr_dst, acc, x, y,
                                   any_band(c));
}

// ---------------------------------------------------------------------------
// K steps per sweep through LDS (K = 2 or 3).  A tile of w x h nodes
// (w <= TW, h <= TH) at (x0, y0) is advanced K steps by updates over
// shrinking regions: R_j is the tile grown by a ring of j nodes (clipped to
// the cavity; unwrapped coordinates across a periodic seam).  The first
// update advances R_(K-1) from the global state into LDS, each middle update
// advances R_j (j = K-2 .. 1) in place in LDS (every node first reads its
// pulls into registers, then, after a barrier, writes its own slot), and the
// last update advances the tile from LDS into the global state.  The
// intermediate populations are kept in their storage type, so the result is
// bit-identical to K single steps.  The state crosses HBM once per K steps.
// A wall node pulls through its partner from at most one node beyond it
// inward, so R_j covers the update of R_(j-1) as long as no tile starts on
// the last column or row of a cavity (the host's tiling guarantees it).
// Only the tile's own nodes write wall tallies.  Plain layouts and the FP32
// layout with the FP64 rest enthalpy population: the LDS holds each
// population in the type it is stored in.
// ---------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__)
#define LBM_HOST_CHECK(cond) ((void)0)
#else
#define LBM_HOST_CHECK(cond)                                                              \
    do {                                                                                  \
        if (!(cond)) {                                                                    \
            fprintf(stderr, "lbm: check failed: %s (%s:%d)\n", #cond, __FILE__, __LINE__); \
            abort();                                                                      \
        }                                                                                 \
    } while (0)
#endif

// How a layout keeps its populations in LDS for the K-step kernels: encoded
// exactly as it stores them (element type, 16-bit scale, split base), so
// that the next update sees the same values as a one-step launch would
// load.  put_node writes a node's post-collision offsets and the split
// layout's base values (bf, bg, bh, as the stores take them); get returns
// one population as the layout's load does.  NSLOT is the plane stride.
template <class Lay>
struct LdsCodec;
template <class E, bool SCALED, int QT_>
struct LdsCodec<Plain<E, SCALED, QT_>> {
    using T = typename E::T;
    using C = decltype(E::dec(T()));
    static constexpr int QT = QT_;
    static constexpr size_t bytes(int nslot) { return (size_t)(9 + 2 * QT) * nslot * sizeof(T); }
    LBM_HD static int plane(int f, int i) { return f == 0 ? i : 9 + (f - 1) * QT + i; }
    template <typename V, typename R>
    LBM_HD static void put1(void *lds, int nslot, int f, int i, int slot, V v, const CavityConst<R> &c) {
        ((T *)lds)[plane(f, i) * nslot + slot] = E::enc((C)(SCALED ? v * (V)c.scale[f] : v));
    }
    template <typename R, typename RH>
    LBM_HD static void put_node(void *lds, int nslot, int slot, const CavityConst<R> &c, const R qf[9],
                                const RH qg[9], const R qh[9], R bf, RH bg, R bh) {
        (void)bf;
        (void)bg;
        (void)bh;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            put1(lds, nslot, 0, i, slot, qf[i], c);
            if (i < QT) {
                put1(lds, nslot, 1, i, slot, qg[i], c);
                put1(lds, nslot, 2, i, slot, qh[i], c);
            }
        }
    }
    template <typename V, typename R>
    LBM_HD static V get(const void *lds, int nslot, int f, int i, int slot, const CavityConst<R> &c) {
        const V v = (V)E::dec(((const T *)lds)[plane(f, i) * nslot + slot]);
        return SCALED ? v * (V)c.inv_scale[f] : v;
    }
};
template <int QT_>
struct LdsCodec<PlainH64<QT_>> {
    static constexpr int QT = QT_;
    static constexpr int NF32 = PlainH64<QT_>::NF32;
    // FP32 planes, then the FP64 rest enthalpy plane (8-byte aligned)
    static constexpr size_t f64_offset(int nslot) { return ((size_t)NF32 * nslot * 4 + 7) & ~(size_t)7; }
    static constexpr size_t bytes(int nslot) { return f64_offset(nslot) + (size_t)nslot * 8; }
    template <typename V>
    LBM_HD static void put1(void *lds, int nslot, int f, int i, int slot, V v) {
        if (f == 1 && i == 0) ((double *)((char *)lds + f64_offset(nslot)))[slot] = (double)v;
        else ((float *)lds)[PlainH64<QT_>::plane(f, i) * nslot + slot] = (float)v;
    }
    template <typename V, typename R>
    LBM_HD static void put1(void *lds, int nslot, int f, int i, int slot, V v, const CavityConst<R> &c) {
        (void)c;
        put1(lds, nslot, f, i, slot, v);
    }
    template <typename R, typename RH>
    LBM_HD static void put_node(void *lds, int nslot, int slot, const CavityConst<R> &c, const R qf[9],
                                const RH qg[9], const R qh[9], R bf, RH bg, R bh) {
        (void)c;
        (void)bf;
        (void)bg;
        (void)bh;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            put1(lds, nslot, 0, i, slot, qf[i]);
            if (i < QT) {
                put1(lds, nslot, 1, i, slot, qg[i]);
                put1(lds, nslot, 2, i, slot, qh[i]);
            }
        }
    }
    template <typename V, typename R>
    LBM_HD static V get(const void *lds, int nslot, int f, int i, int slot, const CavityConst<R> &c) {
        (void)c;
        if (f == 1 && i == 0) return (V)((const double *)((const char *)lds + f64_offset(nslot)))[slot];
        return (V)((const float *)lds)[PlainH64<QT_>::plane(f, i) * nslot + slot];
    }
};
// Split 16-bit layout: per field the FP32 rest population and base, then the
// eight 16-bit remainders from the base's rest equilibrium.
template <class ER>
struct LdsCodec<SplitT<ER>> {
    static constexpr int QT = 9;
    static constexpr size_t bytes(int nslot) { return (size_t)nslot * (6 * 4 + 24 * 2); }
    template <typename V, typename R>
    LBM_HD static void put_field(void *lds, int nslot, int f, int slot, const V q[9], V beta,
                                 const CavityConst<R> &c) {
        float *P = (float *)lds;
        uint16_t *Qp = (uint16_t *)(P + 6 * nslot);
        const float b = (float)split_base<V>(beta);
        P[(2 * f) * nslot + slot] = (float)q[0];
        P[(2 * f + 1) * nslot + slot] = b;
#pragma unroll
        for (int i = 1; i < 9; ++i)
            Qp[(8 * f + i - 1) * nslot + slot] = ER::enc(split_rem<V>(i, q[i], (V)b, (V)c.scale[f]));
    }
    template <typename R, typename RH>
    LBM_HD static void put_node(void *lds, int nslot, int slot, const CavityConst<R> &c, const R qf[9],
                                const RH qg[9], const R qh[9], R bf, RH bg, R bh) {
        put_field(lds, nslot, 0, slot, qf, bf, c);
        put_field(lds, nslot, 1, slot, qg, bg, c);
        put_field(lds, nslot, 2, slot, qh, bh, c);
    }
    template <typename V, typename R>
    LBM_HD static V get(const void *lds, int nslot, int f, int i, int slot, const CavityConst<R> &c) {
        const float *P = (const float *)lds;
        if (i == 0) return (V)P[(2 * f) * nslot + slot];
        const V b = (V)P[(2 * f + 1) * nslot + slot];
        const uint16_t *Qp = (const uint16_t *)(P + 6 * nslot);
        const V r = (V)ER::dec(Qp[(8 * f + i - 1) * nslot + slot]);
        return split_dec<V>(i, b, r, (V)c.inv_scale[f]);
    }
};

// LDS placement of the intermediate populations.  Pull placement: a node
// writes its post-collision populations to its own slot and the next update
// reads each pull from the neighbour's slot, so the planes cover the first
// update's whole region.  Push placement: a node writes population i to the
// slot of the node that pulls it (x + e_i) and the next update reads all of
// its pulls from its own slot, so the planes need only cover the nodes that
// later updates read, the tile grown by K - 2 nodes; writes that fall
// outside are dropped.  Push is chosen where the smaller planes let one more
// workgroup share a CU.
#ifndef LBM_PUSH_F32_K3
#define LBM_PUSH_F32_K3 1
#endif
template <class Lay, int K>
struct PushLds {
    static constexpr bool value = false;
};
template <>
struct PushLds<Plain<E32, false, 9>, 3> {
    static constexpr bool value = LBM_PUSH_F32_K3;
};
#ifndef LBM_PUSH_F32H_K3
#define LBM_PUSH_F32H_K3 1
#endif
template <>
struct PushLds<PlainH64<9>, 3> {
    static constexpr bool value = LBM_PUSH_F32H_K3;
};
#ifndef LBM_PUSH_F64_K2
#define LBM_PUSH_F64_K2 1
#endif
template <>
struct PushLds<Plain<E64, false, 9>, 2> {
    static constexpr bool value = LBM_PUSH_F64_K2;
};

template <class Lay>
struct IsSplitLayout {
    static constexpr bool value = false;
};
template <class ER>
struct IsSplitLayout<SplitT<ER>> {
    static constexpr bool value = true;
};

template <class Lay, int TW, int TH, int K>
struct StepKShape {
    static constexpr int QT = Lay::QT;
    static constexpr int RING = K - 1;          // ring of the first update
    static constexpr int LW = TW + 2 * RING;    // thread map pitch of the first update
    static constexpr int NFIRST = LW * (TH + 2 * RING);  // threads of the first update
    static constexpr bool PUSH = PushLds<Lay, K>::value;
    static constexpr int WR = PUSH ? K - 2 : RING;       // ring of the LDS window
    static constexpr int WW = TW + 2 * WR, WH = TH + 2 * WR;  // LDS window
    static constexpr int NSLOT = WW * WH;                // LDS plane stride
    using Codec = LdsCodec<Lay>;
    static constexpr size_t LDS_BYTES = Codec::bytes(NSLOT);
    // Split layouts: every pull of the first update needs the base of the
    // node it pulls from, so the workgroup first copies the bases of the
    // pulled region (the first update's region and one more ring) into LDS
    // and the pulls read them there instead of loading one base per pull.
    static constexpr bool STAGE_BASE = IsSplitLayout<Lay>::value;
    static constexpr int BW = TW + 2 * K, BH = TH + 2 * K;  // pulled region
    static constexpr int BP = BW;  // row pitch of the staged bases
    static constexpr int NBASE = STAGE_BASE ? BP * BH : 0;   // base plane stride
    static constexpr size_t BASE_BYTES = (size_t)3 * NBASE * sizeof(float);
    static_assert(TH + 2 * K <= LBM_MIN_BAND_ROWS, "a tile's rows must span at most two bands");
};

// Global accesses of a tile go through 32-bit offsets from the block of the
// band of the first row any update touches, y0 - K (the first update's ring
// and its pulls), clipped to the cavity: at most TH + 2K <= LBM_MIN_BAND_ROWS
// rows, so at most two bands.
template <typename R, int K>
LBM_HD int tile_first_row(const CavityConst<R> &c, const Tile2 &tl) {
    (void)c;
    return tl.y0 >= K ? tl.y0 - K : 0;
}

// LDS slot of the node at unwrapped (x, y) of a tile's K-step sweep.
template <class Sh>
LBM_HD int lds_slot(const Tile2 &tl, int x, int y) {
    return (y - (tl.y0 - Sh::WR)) * Sh::WW + (x - (tl.x0 - Sh::WR));
}

// Push placement: population i of the node at unwrapped (x, y) goes to the
// slot of x + e_i if that lies in the window; Sr_f to the node's own slot.
template <class Sh, typename R, typename RH>
LBM_HD void lds_push(const CavityConst<R> &c, const Tile2 &tl, int x, int y, void *lds_q, R *lds_sr, const R qf[9],
                     const RH qg[9], const R qh[9], RH srf) {
    using Cd = typename Sh::Codec;
    const int wx = x - (tl.x0 - Sh::WR), wy = y - (tl.y0 - Sh::WR);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int dx = wx + ex_of(i), dy = wy + ey_of(i);
        if (dx >= 0 && dx < Sh::WW && dy >= 0 && dy < Sh::WH) {
            const int sl = dy * Sh::WW + dx;
            LBM_HOST_CHECK(sl >= 0 && sl < Sh::NSLOT);
            Cd::put1(lds_q, Sh::NSLOT, 0, i, sl, qf[i], c);
            if (i < Sh::QT) {
                Cd::put1(lds_q, Sh::NSLOT, 1, i, sl, qg[i], c);
                Cd::put1(lds_q, Sh::NSLOT, 2, i, sl, qh[i], c);
            }
        }
    }
    if (wx >= 0 && wx < Sh::WW && wy >= 0 && wy < Sh::WH) lds_sr[wy * Sh::WW + wx] = (R)srf;
}

// Split layouts, before the first update: thread t (of NT) copies the
// bases of its nodes of the pulled region (unwrapped columns tl.x0 - K ..
// tl.x0 + w + K - 1, rows tl.y0 - K .. tl.y0 + h + K - 1, at row pitch BP;
// nodes outside the cavity are skipped, nothing reads them) into three LDS
// planes of NBASE.
template <class Lay, typename R, int TW, int TH, int K, int NT>
LBM_HD void stepk_stage_bases(const CavityConst<R> &c, const Tile2 &tl, const void *src, float *lds_b, int t) {
    using Sh = StepKShape<Lay, TW, TH, K>;
    static_assert(Sh::STAGE_BASE, "split layouts only");
    const int yb = tile_first_row<R, K>(c, tl);
    const BandOrigin org = band_origin(c, yb);
    const void *blk = band_block(c, src, yb / c.band_rows);
    const int64_t stride = c.band_nodes;
    for (int q = t; q < Sh::BP * (tl.h + 2 * K); q += NT) {
        const int bx = q % Sh::BP;
        if (bx >= tl.w + 2 * K) continue;
        const int x = tl.x0 - K + bx, y = tl.y0 - K + q / Sh::BP;  // unwrapped
        if (y < 0 || y >= c.ny) continue;
        int xx = x;
        if (c.periodic) xx = x < 0 ? x + c.nx : (x >= c.nx ? x - c.nx : x);
        else if (x < 0 || x >= c.nx) continue;
        LBM_HOST_CHECK(xx >= 0 && xx < c.nx && q < Sh::NBASE);
        LBM_HOST_CHECK(y >= yb && y < yb + TH + 2 * K && y < org.y_next + c.band_rows);
        const NodeRef k = org(xx, y);
#pragma unroll
        for (int f = 0; f < 3; ++f) lds_b[f * Sh::NBASE + q] = Lay::load_base(blk, stride, f, k);
    }
}

// Split layouts, first update: the pulls of the node at unwrapped column x
// (wrapped xx) or of its wall partner, with the pulled nodes' bases from
// the staged LDS copy; the same values as gather_at.
template <class Lay, typename R, typename RH, int TW, int TH, int K>
LBM_HD void gather_staged(const CavityConst<R> &c, const Tile2 &tl, const void *blk, const NodeGeom &g, int x,
                          int xx, const BandOrigin &org, const float *lds_b, R qf[9], RH qg[9], R qh[9]) {
    using Sh = StepKShape<Lay, TW, TH, K>;
    const int64_t stride = c.band_nodes;
    const int px = x + (g.sx - xx);  // partner column, unwrapped
    const NodeRef rows[3] = {org.row(g.sy - 1), org.row(g.sy), org.row(g.sy + 1)};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int sx = g.sx - ex_of(i);
        if (c.periodic) sx = sx < 0 ? sx + c.nx : (sx >= c.nx ? sx - c.nx : sx);
        const NodeRef k = BandOrigin::at_row(rows[1 - ey_of(i)], sx);
        if (i == 0) {
            qf[0] = Lay::template load<R>(blk, stride, 0, 0, k, c);
            qg[0] = Lay::template load<RH>(blk, stride, 1, 0, k, c);
            qh[0] = Lay::template load<R>(blk, stride, 2, 0, k, c);
            continue;
        }
        const int bi = (g.sy - ey_of(i) - (tl.y0 - K)) * Sh::BP + (px - ex_of(i) - (tl.x0 - K));
        LBM_HOST_CHECK(px - ex_of(i) - (tl.x0 - K) >= 0 && px - ex_of(i) - (tl.x0 - K) < tl.w + 2 * K);
        LBM_HOST_CHECK(g.sy - ey_of(i) - (tl.y0 - K) >= 0 && g.sy - ey_of(i) - (tl.y0 - K) < tl.h + 2 * K);
        LBM_HOST_CHECK(bi >= 0 && bi < Sh::NBASE);
        qf[i] = Lay::template load_moving<R>(blk, stride, 0, i, k, (R)lds_b[bi], c);
        qg[i] = Lay::template load_moving<RH>(blk, stride, 1, i, k, (RH)lds_b[Sh::NBASE + bi], c);
        qh[i] = Lay::template load_moving<R>(blk, stride, 2, i, k, (R)lds_b[2 * Sh::NBASE + bi], c);
    }
}

// First update: slot s of R_(K-1) (row-major with the fixed pitch LW, so the
// decode divides by a constant; columns beyond w + 2 RING idle).  Reads the
// global state (split layouts: with the bases staged in lds_b), writes the
// slot's post-collision populations and Sr_f to LDS.
template <class Lay, typename R, typename RH, int TW, int TH, int K>
LBM_HD void stepk_first(const CavityConst<R> &c, const Tile2 &tl, const void *src,
                        const R *__restrict__ sr_src, double *__restrict__ acc, void *lds_q, R *lds_sr,
                        const float *lds_b, int s) {
    using Sh = StepKShape<Lay, TW, TH, K>;
    constexpr int LW = Sh::LW, RG = Sh::RING;
    LBM_HOST_CHECK(s >= 0 && s < LW * (tl.h + 2 * RG) && s < Sh::NFIRST);
    const int lx = s % LW, ly = s / LW;
    if (lx >= tl.w + 2 * RG) return;
    const int x = tl.x0 - RG + lx, y = tl.y0 - RG + ly;  // unwrapped
    if (y < 0 || y >= c.ny) return;
    int xx = x;
    if (c.periodic) xx = x < 0 ? x + c.nx : (x >= c.nx ? x - c.nx : x);
    else if (x < 0 || x >= c.nx) return;
    LBM_HOST_CHECK(xx >= 0 && xx < c.nx);
    const bool owned = x >= tl.x0 && x < tl.x0 + tl.w && y >= tl.y0 && y < tl.y0 + tl.h;
    const NodeGeom g = geometry(c, xx, y, true);
    const int yb = tile_first_row<R, K>(c, tl);
    const BandOrigin org = band_origin(c, yb);
    LBM_HOST_CHECK(g.sy - 1 >= yb && g.sy + 1 < yb + TH + 2 * K);
    LBM_HOST_CHECK(g.sy + 1 < org.y_next + c.band_rows);
    R qf[9], qh[9];
    RH qg[9];
    if constexpr (Sh::STAGE_BASE)
        gather_staged<Lay, R, RH, TW, TH, K>(c, tl, band_block(c, src, yb / c.band_rows), g, x, xx, org, lds_b, qf,
                                              qg, qh);
    else
        gather_at<Lay, R, RH, true>(c, band_block(c, src, yb / c.band_rows), g, xx, y, org, qf, qg, qh);
    (void)lds_b;
    Thermo<RH> th;
    Macro<R> m;
    const R sr_prev = sr_src[flat_index(c, xx, y)];
    const RH srf = update_node<Sh::QT, R, RH, true>(c, g, xx, y, qf, qg, qh, sr_prev, owned, acc, th, m);
    if constexpr (Sh::PUSH) {
        lds_push<Sh, R, RH>(c, tl, x, y, lds_q, lds_sr, qf, qg, qh, srf);
    } else {
        const ThermalConst<RH> &t = thermal<RH>(c);
        Sh::Codec::put_node(lds_q, Sh::NSLOT, s, c, qf, qg, qh, m.drho, t.c_fref * (th.Tf - t.T_ref),
                            c.c_mref * m.dTm);
        lds_sr[s] = (R)srf;
    }
}

// A node's pulls from LDS: the slots of the neighbours of the node (or of
// its wall partner), in unwrapped coordinates.  x is the node's unwrapped
// column, xx the wrapped one.
template <class Sh, typename R, typename RH>
LBM_HD void lds_gather(const CavityConst<R> &c, const Tile2 &tl, const NodeGeom &g, int x, int xx, int h_region,
                       const void *lds_q, R qf[9], RH qg[9], R qh[9]) {
    using Cd = typename Sh::Codec;
    const int px = x + (g.sx - xx);  // partner column, unwrapped
    if constexpr (Sh::PUSH) {
        // every pull of the node (or of its partner) sits in its own slot
        const int sl = lds_slot<Sh>(tl, px, g.sy);
        LBM_HOST_CHECK(px - (tl.x0 - Sh::WR) >= 0 && px - (tl.x0 - Sh::WR) < Sh::WW);
        LBM_HOST_CHECK(g.sy - (tl.y0 - Sh::WR) >= 0 && g.sy - (tl.y0 - Sh::WR) < Sh::WH);
        LBM_HOST_CHECK(sl >= 0 && sl < Sh::NSLOT);
        (void)h_region;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            qf[i] = Cd::template get<R>(lds_q, Sh::NSLOT, 0, i, sl, c);
            if (i < Sh::QT) {
                qg[i] = Cd::template get<RH>(lds_q, Sh::NSLOT, 1, i, sl, c);
                qh[i] = Cd::template get<R>(lds_q, Sh::NSLOT, 2, i, sl, c);
            } else {
                qg[i] = RH(0);
                qh[i] = R(0);
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int sl = lds_slot<Sh>(tl, px - ex_of(i), g.sy - ey_of(i));
        LBM_HOST_CHECK(px - ex_of(i) - (tl.x0 - Sh::RING) >= 0 && px - ex_of(i) - (tl.x0 - Sh::RING) < Sh::LW);
        LBM_HOST_CHECK(g.sy - ey_of(i) - (tl.y0 - Sh::RING) >= 0 &&
                       g.sy - ey_of(i) - (tl.y0 - Sh::RING) < h_region);
        LBM_HOST_CHECK(sl >= 0 && sl < Sh::NSLOT);
        qf[i] = Cd::template get<R>(lds_q, Sh::NSLOT, 0, i, sl, c);
        if (i < Sh::QT) {
            qg[i] = Cd::template get<RH>(lds_q, Sh::NSLOT, 1, i, sl, c);
            qh[i] = Cd::template get<R>(lds_q, Sh::NSLOT, 2, i, sl, c);
        } else {
            qg[i] = RH(0);
            qh[i] = R(0);
        }
    }
}

// A middle update of ring j (1 <= j <= K - 2), split at the barrier that
// lets it run in place: stepk_mid_load reads thread t's node's pulls into
// registers (false: the thread has no node), stepk_mid_store updates the
// node and writes its own slot.
template <typename R, typename RH>
struct MidNode {
    int x, xx, y, slot;
    bool owned;
    NodeGeom g;
    R qf[9], qh[9], sr_prev;
    RH qg[9];
};
template <class Lay, typename R, typename RH, int TW, int TH, int K>
LBM_HD bool stepk_mid_load(const CavityConst<R> &c, const Tile2 &tl, int j, const void *lds_q, const R *lds_sr,
                           int t, MidNode<R, RH> &n) {
    using Sh = StepKShape<Lay, TW, TH, K>;
    const int pw = TW + 2 * j;  // pitch of ring j's thread map
    const int lx = t % pw, ly = t / pw;
    if (lx >= tl.w + 2 * j || ly >= tl.h + 2 * j) return false;
    n.x = tl.x0 - j + lx;
    n.y = tl.y0 - j + ly;  // unwrapped
    if (n.y < 0 || n.y >= c.ny) return false;
    n.xx = n.x;
    if (c.periodic) n.xx = n.x < 0 ? n.x + c.nx : (n.x >= c.nx ? n.x - c.nx : n.x);
    else if (n.x < 0 || n.x >= c.nx) return false;
    LBM_HOST_CHECK(n.xx >= 0 && n.xx < c.nx);
    n.owned = n.x >= tl.x0 && n.x < tl.x0 + tl.w && n.y >= tl.y0 && n.y < tl.y0 + tl.h;
    n.g = geometry(c, n.xx, n.y, true);
    n.slot = lds_slot<Sh>(tl, n.x, n.y);
    LBM_HOST_CHECK(n.slot >= 0 && n.slot < Sh::NSLOT);
    lds_gather<Sh, R, RH>(c, tl, n.g, n.x, n.xx, tl.h + 2 * Sh::RING, lds_q, n.qf, n.qg, n.qh);
    n.sr_prev = lds_sr[n.slot];
    return true;
}
template <class Lay, typename R, typename RH, int TW, int TH, int K>
LBM_HD void stepk_mid_store(const CavityConst<R> &c, const Tile2 &tl, double *__restrict__ acc, void *lds_q,
                            R *lds_sr, MidNode<R, RH> &n) {
    using Sh = StepKShape<Lay, TW, TH, K>;
    Thermo<RH> th;
    Macro<R> m;
    const RH srf = update_node<Sh::QT, R, RH, true>(c, n.g, n.xx, n.y, n.qf, n.qg, n.qh, n.sr_prev, n.owned, acc,
                                                   th, m);
    if constexpr (Sh::PUSH) {
        lds_push<Sh, R, RH>(c, tl, n.x, n.y, lds_q, lds_sr, n.qf, n.qg, n.qh, srf);
    } else {
        const ThermalConst<RH> &t = thermal<RH>(c);
        Sh::Codec::put_node(lds_q, Sh::NSLOT, n.slot, c, n.qf, n.qg, n.qh, m.drho, t.c_fref * (th.Tf - t.T_ref),
                            c.c_mref * m.dTm);
        lds_sr[n.slot] = (R)srf;
    }
}

// Last update: node n of the tile (row-major with pitch TW; columns beyond
// w idle).  Pulls from LDS, writes the global state.
template <class Lay, typename R, typename RH, int TW, int TH, int K>
LBM_HD void stepk_last(const CavityConst<R> &c, const Tile2 &tl, void *dst, R *__restrict__ sr_dst,
                       double *__restrict__ acc, const void *lds_q, const R *lds_sr, int n) {
    using Sh = StepKShape<Lay, TW, TH, K>;
    LBM_HOST_CHECK(n >= 0 && n < TW * tl.h);
    if (n % TW >= tl.w) return;
    const int x = tl.x0 + n % TW, y = tl.y0 + n / TW;
    LBM_HOST_CHECK(x >= 0 && x < c.nx && y >= 0 && y < c.ny);
    const NodeGeom g = geometry(c, x, y, true);
    R qf[9], qh[9];
    RH qg[9];
    lds_gather<Sh, R, RH>(c, tl, g, x, x, tl.h + 2 * Sh::RING, lds_q, qf, qg, qh);
    const int self = lds_slot<Sh>(tl, x, y);
    const int yb = tile_first_row<R, K>(c, tl);
    const NodeRef k = band_origin(c, yb)(x, y);
    void *blk = band_block(c, dst, yb / c.band_rows);
    Thermo<RH> th;
    Macro<R> m;
    const RH srf = update_node<Sh::QT, R, RH, true>(c, g, x, y, qf, qg, qh, lds_sr[self], true, acc, th, m);
    const ThermalConst<RH> &t = thermal<RH>(c);
    const int64_t stride = c.band_nodes;
    Lay::template store<R>(blk, stride, 0, qf, m.drho, k, c);
    Lay::template store<RH>(blk, stride, 1, qg, t.c_fref * (th.Tf - t.T_ref), k, c);
    Lay::template store<R>(blk, stride, 2, qh, c.c_mref * m.dTm, k, c);
    sr_dst[flat_index(c, x, y)] = (R)srf;
}

// Macroscopic fields of one node (post-streaming state) plus its
// contributions to the diagnostics partial sums.
template <class Lay, typename R, typename RH>
LBM_HD void macro_node(const CavityConst<R> &c, const void *src, bool raw, int x, int y, double out[6],
                       double v[NPART]) {
    const int nx = c.nx, ny = c.ny;
    const NodeGeom g = geometry(c, x, y, !raw);
    R qf[9], qh[9];
    RH qg[9];
    if (raw) gather<Lay, R, RH, false>(c, src, g, x, y, qf, qg, qh);
    else gather<Lay, R, RH, true>(c, src, g, x, y, qf, qg, qh);
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        finite = finite && isfinite(qf[i]) && (i >= Lay::QT || (isfinite(qg[i]) && isfinite(qh[i])));
    // inflow of the last step through the wall links (not yet tallied)
    if (!raw && !g.wall) {
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int px = x - ex_of(i), py = y - ey_of(i);
            const bool onx = !c.periodic && (px == 0 || px == nx - 1);
            const bool ony = (py == 0 || py == ny - 1);
            if (onx || ony) {
                const int w = onx ? (px == 0 ? W_LEFT : W_RIGHT) : (py == 0 ? W_BOTTOM : W_TOP);
                double e, mm;
                link_content<Lay::QT>(c, i, qf, qg, qh, e, mm);
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
    if (!raw && g.wall) reconstruct_wall<Lay::QT>(c, x, y, qf, qg, qh);
    double sg = 0.0, sh = 0.0, sf = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (i < Lay::QT) {
            sg += c.g_ref[i] + (double)qg[i];
            sh += c.h_ref[i] + (double)qh[i];
        }
        sf += (double)w_of<double>(i) + (double)qf[i];
    }
    Thermo<RH> th;
    Macro<R> m;
    macros<Lay::QT>(c, qf, qg, qh, th, m);
    out[0] = (double)m.ux;
    out[1] = (double)m.uy;
    out[2] = (double)th.Tf;
    out[3] = (double)m.Tm;
    out[4] = (double)th.fl;
    out[5] = (double)m.rho;
    if (!finite) v[P_NF] = 1.0;
    if (!g.wall) {
        v[P_FL] = (double)th.fl;
        // phi rho_l H + (1-phi) rho_m c_pm T_m and rho, from the offsets
        v[P_E] = c.we * sg + c.wm * sh;
        v[P_M] = sf;
        v[P_DT] = fabs((double)th.Tf - (double)m.Tm);
        v[P_U] = sqrt((double)m.ux * (double)m.ux + (double)m.uy * (double)m.uy);
    }
}

// Initial state of one node: equilibria at rest (Eqs. 27, 40, 49) at the
// given temperatures, stored as offsets; the previous-step source equals the
// current one.
template <class Lay, typename R, typename RH>
LBM_HD void init_node(const CavityConst<R> &c, void *dst, R *sr, int x, int y, double Tf, double Tm) {
    const ThermalConst<double> &t = c.td;
    const int nx = c.nx;
    const bool wall = (!c.periodic && (x == 0 || x == nx - 1)) || y == 0 || y == c.ny - 1;
    const int w = wall ? thermal_wall(c, x, y) : -1;
    if (w >= 0) Tf = Tm = t.T_wall[w];
    // inverse of Eq. (38) (a tie at the solidus goes to the solid branch)
    double H;
    if (Tf <= t.T_fs) H = Tf / t.inv_cps;
    else if (Tf >= t.T_fl) H = (Tf - t.T_fl) / t.inv_cpl + t.H_fl;
    else H = t.H_fs + (Tf - t.T_fs) / (t.T_fl - t.T_fs) * (t.H_fl - t.H_fs);
    const double dT = Tf - t.T_ref, dTm = Tm - t.T_ref;
    const double dH = H - t.H_ref;
    const double cf = t.c_fref, cm = c.c_mref, cpm = c.c_pm;
    // equilibria at rest, Eqs. (40), (49) / Eqs. (B3), (B5): the moving
    // weights are w_i (D2Q9) or varpi/4 (D2Q5), the rest one takes the rest
    const int QT = Lay::QT;
    const double wrest = QT == 9 ? 5.0 / 9.0 : t.varpi;
    R qf[9], qh[9];
    RH qg[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double wi = QT == 9 ? w_of<double>(i) : 0.25 * t.varpi;
        qf[i] = R(0);
        qg[i] = (RH)(i == 0 ? dH - wrest * cf * dT : wi * cf * dT);
        qh[i] = (R)(i == 0 ? (cpm - wrest * cm) * dTm : wi * cm * dTm);
    }
    const FarRef k = any_band(c)(x, y);
    void *blk = band_block(c, dst, 0);
    const int64_t stride = c.band_nodes;
    Lay::template store<R>(blk, stride, 0, qf, R(0), k, c);
    Lay::template store<RH>(blk, stride, 1, qg, (RH)(cf * dT), k, c);
    Lay::template store<R>(blk, stride, 2, qh, (R)(cm * dTm), k, c);
    sr[flat_index(c, x, y)] = (R)((double)c.hv_f * (Tm - Tf));
}

}  // namespace lbm
