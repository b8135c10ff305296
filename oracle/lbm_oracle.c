/*
 * Plain FP64 CPU oracle for the enthalpy-based multiple-relaxation-time
 * lattice Boltzmann method for solid-liquid phase change in metal foams under
 * local thermal non-equilibrium (Liu, He & Li, arXiv:1701.00702).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, literal oracle that the
 * GPU library is compared against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header or
 * table with the GPU library.
 *
 * Style: one node at a time, dense 9x9 transforms (Eq. 13 and its numerical
 * inverse), every quantity in the order the paper introduces it.  No fusion,
 * no blocking, no offsets.  OpenMP only splits independent node loops.
 *
 * Time step t -> t+1 as implemented here (state = post-streaming populations
 * f+, g, h at every node with the wall nodes already reconstructed, plus the
 * previous-step interstitial sources):
 *   1. macroscopic values from the post-streaming populations:
 *      H (Eq. 37), T_f and f_l (Eqs. 38-39), T_m (Eq. 48), rho (Eq. 21),
 *      volumetric blend (Eq. 20), buoyancy (Eq. 7), velocity (Eqs. 23-25),
 *      total force (Eq. 3);
 *   2. flow collision in moment space (Eqs. 14, 16-19);
 *   3. interstitial sources with the backward difference of Remark III
 *      (Eqs. 36, 47);
 *   4. PCM-enthalpy and metal-foam collisions (Eqs. 32, 34-35 and 43, 45-46);
 *   5. streaming (Eqs. 15, 33, 44);
 *   6. non-equilibrium extrapolation on the wall nodes (Eq. 52 and its thermal
 *      analogues), using the partner node's new populations.
 * Wall fluxes for the energy/mass balance are tallied between 4 and 5.
 *
 * Readings where the paper is silent: walls sit on the first/last node rows and columns and
 * L = nx - 1; the extrapolation partner is the inward normal neighbour (the
 * diagonal one at corners) for all nine directions; corners take the
 * isothermal value of their vertical wall; adiabatic walls copy the partner's
 * temperature; the source derivative is zero at the first step; the
 * liquid fraction of the current step enters the blend and the buoyancy.
 *
 * Variants of the thermal fields: the D2Q9 MRT models of Sec. III B/C, the
 * D2Q5 MRT models of Appendix B (Eqs. B1-B5, weight parameter varpi), and,
 * through the relaxation-rate tables the caller passes, the BGK thermal
 * models of Sec. V A (every rate 1/tau) and other zeta_e values (Sec. V D).
 * Each wall is isothermal at a given temperature or adiabatic; at a corner
 * an isothermal vertical wall wins, then an isothermal horizontal wall.
 *
 * Solid treatment: the volumetric scheme of Eq. (20), or the bounce-back
 * alternative compared in Sec. V B: a node with f_l < 0.5 (the interface
 * is f_l = 0.5) is solid, its flow populations are reflected
 * (f*_i = f+_{-i}) and its velocity is zero; other nodes collide their
 * unblended f+ with the force of Eq. (3).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

/* D2Q9 velocities, Eq. (11) with c = 1. */
static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Weights listed after Eq. (27). */
static const double WT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* Transformation matrix, Eq. (13). */
static const double MM[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

/* D2Q5 transformation matrix, Eq. (B1); its velocities are the first five
 * of Eq. (11). */
#define Q5 5
static const double M5[Q5][Q5] = {
    {1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0},
    {0, 0, 1, 0, -1},
    {0, 1, 1, 1, 1},
    {0, 1, -1, 1, -1},
};

enum { W_NONE = -1, W_LEFT = 0, W_RIGHT = 1, W_BOTTOM = 2, W_TOP = 3 };
enum { WALL_ISOTHERMAL = 1, WALL_ADIABATIC = 2 };
/* Opposite direction of each D2Q9 velocity. */
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

typedef struct {
    /* geometry: a window [gx0, gx0+nx) x [gy0, gy0+ny) of an NX x NY cavity */
    int nx, ny, gx0, gy0, NX, NY;
    int periodic_x;   /* 1: periodic in x, no vertical walls */
    int gravity_axis; /* 1: gravity along -y, 0: along -x */
    /* materials and lattice constants */
    double phi, rho_l, rho_m, c_pl, c_ps, c_pm, c_fref, c_mref;
    double nu_f, K, F_phi, gbeta, T0;
    double h_v, L_a, T_fs, T_fl;
    double T_hot, T_cold;
    double k_f, k_m, L; /* diagnostics only: conductivities and length */
    double s[Q];        /* flow relaxation rates, Eq. (16) order */
    double zeta[Q];     /* PCM relaxation rates, Theta in Eq. (31) */
    double eta[Q];      /* metal relaxation rates, Q in Eq. (42) */
    /* thermal lattice: 9 (Sec. III) or 5 (Appendix B; zeta and eta then
     * hold the five rates of Theta and Q in the moment order of Eq. B1) */
    int qt;
    double varpi;       /* D2Q5 weight parameter, Eq. (B2) */
    int wall_type[4];   /* left, right, bottom, top: isothermal or adiabatic */
    double wall_T[4];   /* temperature of the isothermal walls */
    int bounce_back;    /* 0: volumetric scheme (Eq. 20); 1: bounce-back (Sec. V B) */
} oracle_params;

typedef struct {
    double step, Fo, liquid_fraction, Nu_hot, Nu_hot_pcm, Nu_cold;
    double E_int, E_int0, flux_E[4], energy_residual;
    double M_int, M_int0, flux_M[4], mass_residual;
    double x_front_mid, max_dT_LTNE, u_max, nonfinite;
} oracle_diag;

typedef struct {
    double H, T_f, f_l, T_m, rho, ux, uy, Gx, Gy;
    double fb[Q]; /* blended flow populations, Eq. (20) */
} macros;

typedef struct {
    oracle_params p;
    double Minv[Q][Q];
    double M5inv[Q5][Q5];
    double *f, *g, *h;    /* post-streaming state, [node][Q] */
    double *fs, *gs, *hs; /* post-collision populations, [node][Q] */
    double *srf, *srm;    /* previous-step interstitial sources */
    unsigned char *valid, *valid_new;
    long step;
    double flux_E[4], flux_M[4];
    double E0, M0;
} oracle_state;

/* ------------------------------------------------------------------ */
/* Linear algebra: inverse of M by Gauss-Jordan elimination.           */
/* ------------------------------------------------------------------ */
static int invert_n(int n, const double *a_in, double *inv)
{
    double a[Q][2 * Q];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            a[r][c] = c < n ? a_in[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = a[col][c];
                a[col][c] = a[piv][c];
                a[piv][c] = t;
            }
        double d = a[col][col];
        for (int c = 0; c < 2 * n; ++c) a[col][c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double fct = a[r][col];
            if (fct == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) a[r][c] -= fct * a[col][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) inv[r * n + c] = a[r][n + c];
    return 0;
}

static int invert9(const double a_in[Q][Q], double inv[Q][Q])
{
    return invert_n(Q, &a_in[0][0], &inv[0][0]);
}

static int invert5(const double a_in[Q5][Q5], double inv[Q5][Q5])
{
    return invert_n(Q5, &a_in[0][0], &inv[0][0]);
}

static void matvec(const double A[Q][Q], const double *x, double *y)
{
    for (int r = 0; r < Q; ++r) {
        double acc = 0.0;
        for (int c = 0; c < Q; ++c) acc += A[r][c] * x[c];
        y[r] = acc;
    }
}

static void matvec5(const double A[Q5][Q5], const double *x, double *y)
{
    for (int r = 0; r < Q5; ++r) {
        double acc = 0.0;
        for (int c = 0; c < Q5; ++c) acc += A[r][c] * x[c];
        y[r] = acc;
    }
}

/* ------------------------------------------------------------------ */
/* Equilibria in velocity space.                                       */
/* ------------------------------------------------------------------ */

/* Eq. (27): flow equilibrium (alpha1 = 1, alpha2 = -3), c_s^2 = 1/3. */
void oracle_feq(double rho, double ux, double uy, double phi, double *out)
{
    const double cs2 = 1.0 / 3.0;
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < Q; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        out[i] = WT[i] * rho * (1.0 + eu / cs2 + eu * eu / (2.0 * phi * cs2 * cs2) - uu / (2.0 * phi * cs2));
    }
}

/* Eq. (40): PCM enthalpy equilibrium. */
void oracle_geq(double H, double T, double ux, double uy, double phi, double c_fref, double c_pl,
                double *out)
{
    const double cs2 = 1.0 / 3.0;
    out[0] = H - 5.0 / 9.0 * c_fref * T;
    for (int i = 1; i < Q; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        out[i] = WT[i] * c_pl * T * (c_fref / c_pl + eu / (phi * cs2));
    }
}

/* Eq. (49): metal-foam internal-energy equilibrium. */
void oracle_heq(double T_m, double c_pm, double c_mref, double *out)
{
    out[0] = c_pm * T_m - 5.0 / 9.0 * c_mref * T_m;
    for (int i = 1; i < Q; ++i) out[i] = WT[i] * c_mref * T_m;
}

/* Eq. (B3): D2Q5 PCM enthalpy equilibrium, sound speed c_sT^2 = varpi/2. */
void oracle_geq5(double H, double T, double ux, double uy, double phi, double c_fref, double c_pl,
                 double varpi, double *out)
{
    const double cs2 = varpi / 2.0;
    out[0] = H - varpi * c_fref * T;
    for (int i = 1; i < Q5; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        out[i] = 0.25 * varpi * c_pl * T * (c_fref / c_pl + eu / (phi * cs2));
    }
}

/* Eq. (B5): D2Q5 metal-foam internal-energy equilibrium. */
void oracle_heq5(double T_m, double c_pm, double c_mref, double varpi, double *out)
{
    out[0] = c_pm * T_m - varpi * c_mref * T_m;
    for (int i = 1; i < Q5; ++i) out[i] = 0.25 * varpi * c_mref * T_m;
}

/* Thermal equilibria of the configured lattice (unused directions zero). */
static void geq_of(const oracle_params *p, double H, double T, double ux, double uy, double *out)
{
    if (p->qt == Q5) {
        for (int i = Q5; i < Q; ++i) out[i] = 0.0;
        oracle_geq5(H, T, ux, uy, p->phi, p->c_fref, p->c_pl, p->varpi, out);
    } else {
        oracle_geq(H, T, ux, uy, p->phi, p->c_fref, p->c_pl, out);
    }
}

static void heq_of(const oracle_params *p, double T_m, double *out)
{
    if (p->qt == Q5) {
        for (int i = Q5; i < Q; ++i) out[i] = 0.0;
        oracle_heq5(T_m, p->c_pm, p->c_mref, p->varpi, out);
    } else {
        oracle_heq(T_m, p->c_pm, p->c_mref, out);
    }
}

/* Eqs. (38)-(39): temperature and liquid fraction from the enthalpy,
 * branches tested in the order the paper lists them. */
void oracle_eos(const oracle_params *p, double H, double *T, double *fl)
{
    double H_fs = p->c_ps * p->T_fs;
    double H_fl = p->c_pl * p->T_fl + p->L_a;
    if (H <= H_fs) {
        *T = H / p->c_ps;
        *fl = 0.0;
    } else if (H >= H_fl) {
        *T = p->T_fl + (H - H_fl) / p->c_pl;
        *fl = 1.0;
    } else {
        *T = p->T_fs + (H - H_fs) / (H_fl - H_fs) * (p->T_fl - p->T_fs);
        *fl = (H - H_fs) / (H_fl - H_fs);
    }
}

/* Inverse of Eq. (38): enthalpy of a given PCM temperature (a tie at the
 * solidus goes to the solid branch). */
double oracle_enthalpy_of_T(const oracle_params *p, double T)
{
    double H_fs = p->c_ps * p->T_fs;
    double H_fl = p->c_pl * p->T_fl + p->L_a;
    if (T <= p->T_fs) return p->c_ps * T;
    if (T >= p->T_fl) return p->c_pl * (T - p->T_fl) + H_fl;
    return H_fs + (T - p->T_fs) / (p->T_fl - p->T_fs) * (H_fl - H_fs);
}

/* ------------------------------------------------------------------ */
/* Per-node macroscopic values, Eqs. (7), (20)-(25), (37)-(39), (48).  */
/* ------------------------------------------------------------------ */
static void node_macros(const oracle_params *p, const double *fp, const double *g, const double *h,
                        macros *m)
{
    /* Eq. (37) then Eqs. (38)-(39). */
    double H = 0.0;
    for (int i = 0; i < p->qt; ++i) H += g[i];
    m->H = H;
    oracle_eos(p, H, &m->T_f, &m->f_l);
    /* Eq. (48). */
    double eh = 0.0;
    for (int i = 0; i < p->qt; ++i) eh += h[i];
    m->T_m = eh / p->c_pm;
    /* Eq. (21). */
    double rho = 0.0;
    for (int i = 0; i < Q; ++i) rho += fp[i];
    m->rho = rho;
    /* Eq. (20): the solid part is the equilibrium at the solid velocity 0.
     * The bounce-back alternative (Sec. V B) has no blend. */
    double f_solid[Q];
    oracle_feq(rho, 0.0, 0.0, p->phi, f_solid);
    for (int i = 0; i < Q; ++i)
        m->fb[i] = p->bounce_back ? fp[i] : m->f_l * fp[i] + (1.0 - m->f_l) * f_solid[i];
    /* Eq. (7): G = -g beta (T_f - T0) f_l with gravity pointing along -axis. */
    double G = p->gbeta * (m->T_f - p->T0) * m->f_l;
    m->Gx = p->gravity_axis == 0 ? G : 0.0;
    m->Gy = p->gravity_axis == 1 ? G : 0.0;
    /* Eq. (24) with dt = 1. */
    double jx = 0.0, jy = 0.0;
    for (int i = 0; i < Q; ++i) {
        jx += EX[i] * m->fb[i];
        jy += EY[i] * m->fb[i];
    }
    double vx = jx / rho + 0.5 * p->phi * m->Gx;
    double vy = jy / rho + 0.5 * p->phi * m->Gy;
    /* Eq. (25). */
    double l0 = 0.5 * (1.0 + p->phi * 0.5 * p->nu_f / p->K);
    double l1 = p->phi * 0.5 * p->F_phi / sqrt(p->K);
    /* Eq. (23). */
    double vmag = sqrt(vx * vx + vy * vy);
    double den = l0 + sqrt(l0 * l0 + l1 * vmag);
    m->ux = vx / den;
    m->uy = vy / den;
    /* bounce-back: a node below the interface value f_l = 0.5 is solid, at rest */
    if (p->bounce_back && m->f_l < 0.5) {
        m->ux = 0.0;
        m->uy = 0.0;
    }
}

void oracle_node_macros(const oracle_params *p, const double *fp, const double *g, const double *h,
                        double *out9)
{
    macros m;
    node_macros(p, fp, g, h, &m);
    out9[0] = m.H;
    out9[1] = m.T_f;
    out9[2] = m.f_l;
    out9[3] = m.T_m;
    out9[4] = m.rho;
    out9[5] = m.ux;
    out9[6] = m.uy;
    out9[7] = m.Gx;
    out9[8] = m.Gy;
}

/* ------------------------------------------------------------------ */
/* Collision of the three fields at one node.                          */
/* ------------------------------------------------------------------ */

/* D2Q5 thermal collisions of Appendix B: moments by Eq. (B1), equilibrium
 * moments Eqs. (B2) and (B4), sources S (1, 0, 0, varpi, 0), relaxation
 * matrices Theta and Q in the moment order of Eq. (B1). */
static void collide_thermal_d2q5(const oracle_params *p, const double M5inv[Q5][Q5],
                                 const macros *mc, double S_pcm, double S_metal, const double *g,
                                 const double *h, double *go, double *ho)
{
    const double phi = p->phi, vp = p->varpi;
    const double src_dir[Q5] = {1.0, 0.0, 0.0, vp, 0.0};
    double n[Q5], neq[Q5], ns[Q5];
    matvec5(M5, g, n);
    neq[0] = mc->H;
    neq[1] = p->c_pl * mc->T_f * mc->ux / phi;
    neq[2] = p->c_pl * mc->T_f * mc->uy / phi;
    neq[3] = vp * p->c_fref * mc->T_f;
    neq[4] = 0.0;
    for (int k = 0; k < Q5; ++k) ns[k] = n[k] - p->zeta[k] * (n[k] - neq[k]) + S_pcm * src_dir[k];
    matvec5(M5inv, ns, go);
    matvec5(M5, h, n);
    neq[0] = p->c_pm * mc->T_m;
    neq[1] = 0.0;
    neq[2] = 0.0;
    neq[3] = vp * p->c_mref * mc->T_m;
    neq[4] = 0.0;
    for (int k = 0; k < Q5; ++k) ns[k] = n[k] - p->eta[k] * (n[k] - neq[k]) + S_metal * src_dir[k];
    matvec5(M5inv, ns, ho);
    for (int i = Q5; i < Q; ++i) go[i] = ho[i] = 0.0;
}
static void collide_node(const oracle_params *p, const double Minv[Q][Q],
                         const double M5inv[Q5][Q5], const double *fp, const double *g,
                         const double *h, double srf_prev, double srm_prev, double *fo, double *go,
                         double *ho, double *srf_new, double *srm_new)
{
    macros mc;
    node_macros(p, fp, g, h, &mc);
    const double phi = p->phi, rho = mc.rho, ux = mc.ux, uy = mc.uy;
    const double uu = ux * ux + uy * uy;

    /* ---- flow field, Eqs. (14), (16)-(19) ---- */
    /* Eq. (3): total body force. */
    double umag = sqrt(uu);
    double Fx = -phi * p->nu_f / p->K * ux - phi * p->F_phi / sqrt(p->K) * umag * ux + phi * mc.Gx;
    double Fy = -phi * p->nu_f / p->K * uy - phi * p->F_phi / sqrt(p->K) * umag * uy + phi * mc.Gy;
    double m[Q], meq[Q], S[Q], ms[Q];
    matvec(MM, mc.fb, m); /* Eq. (17) */
    /* Eq. (18), alpha1 = 1, alpha2 = -3. */
    meq[0] = rho;
    meq[1] = rho * (-2.0 + 3.0 * uu / phi);
    meq[2] = rho * (1.0 - 3.0 * uu / phi);
    meq[3] = rho * ux;
    meq[4] = -rho * ux;
    meq[5] = rho * uy;
    meq[6] = -rho * uy;
    meq[7] = rho * (ux * ux - uy * uy) / phi;
    meq[8] = rho * ux * uy / phi;
    /* Eq. (19). */
    double uF = ux * Fx + uy * Fy;
    S[0] = 0.0;
    S[1] = rho * 6.0 * uF / phi;
    S[2] = -rho * 6.0 * uF / phi;
    S[3] = rho * Fx;
    S[4] = -rho * Fx;
    S[5] = rho * Fy;
    S[6] = -rho * Fy;
    S[7] = rho * 2.0 * (ux * Fx - uy * Fy) / phi;
    S[8] = rho * (ux * Fy + uy * Fx) / phi;
    /* Eq. (14). */
    for (int k = 0; k < Q; ++k) ms[k] = m[k] - p->s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * p->s[k]) * S[k];
    matvec(Minv, ms, fo); /* f* = M^-1 m*, Eq. (15) */
    /* Sec. V B alternative: a solid node reflects what arrived */
    if (p->bounce_back && mc.f_l < 0.5)
        for (int i = 0; i < Q; ++i) fo[i] = fp[OPP[i]];

    /* ---- interstitial sources, Eqs. (36), (47), Remark III ---- */
    double srf = p->h_v * (mc.T_m - mc.T_f) / (phi * p->rho_l);
    double srm = p->h_v * (mc.T_f - mc.T_m) / ((1.0 - phi) * p->rho_m);
    double S_pcm = srf + 0.5 * (srf - srf_prev);
    double S_metal = srm + 0.5 * (srm - srm_prev);
    *srf_new = srf;
    *srm_new = srm;
    if (p->qt == Q5) {
        collide_thermal_d2q5(p, M5inv, &mc, S_pcm, S_metal, g, h, go, ho);
        return;
    }
    static const double src_dir[Q] = {1, -2, 1, 0, 0, 0, 0, 0, 0}; /* Eqs. (35), (46) */

    /* ---- PCM enthalpy field, Eqs. (32), (34) ---- */
    double n[Q], neq[Q], ns[Q];
    matvec(MM, g, n);
    double T = mc.T_f, H = mc.H;
    neq[0] = H;
    neq[1] = -4.0 * H + 2.0 * p->c_fref * T;
    neq[2] = 4.0 * H - 3.0 * p->c_fref * T;
    neq[3] = p->c_pl * T * ux / phi;
    neq[4] = -p->c_pl * T * ux / phi;
    neq[5] = p->c_pl * T * uy / phi;
    neq[6] = -p->c_pl * T * uy / phi;
    neq[7] = 0.0;
    neq[8] = 0.0;
    for (int k = 0; k < Q; ++k) ns[k] = n[k] - p->zeta[k] * (n[k] - neq[k]) + S_pcm * src_dir[k];
    matvec(Minv, ns, go); /* Eq. (33) */

    /* ---- metal-foam field, Eqs. (43), (45) ---- */
    matvec(MM, h, n);
    double Tm = mc.T_m;
    neq[0] = p->c_pm * Tm;
    neq[1] = -4.0 * p->c_pm * Tm + 2.0 * p->c_mref * Tm;
    neq[2] = 4.0 * p->c_pm * Tm - 3.0 * p->c_mref * Tm;
    for (int k = 3; k < Q; ++k) neq[k] = 0.0;
    for (int k = 0; k < Q; ++k) ns[k] = n[k] - p->eta[k] * (n[k] - neq[k]) + S_metal * src_dir[k];
    matvec(Minv, ns, ho); /* Eq. (44) */
}

void oracle_collide_node(const oracle_params *p, const double *fp, const double *g,
                         const double *h, double srf_prev, double srm_prev, double *fo,
                         double *go, double *ho, double *sr_new2)
{
    double Minv[Q][Q], M5inv[Q5][Q5];
    invert9(MM, Minv);
    invert5(M5, M5inv);
    collide_node(p, Minv, M5inv, fp, g, h, srf_prev, srm_prev, fo, go, ho, &sr_new2[0],
                 &sr_new2[1]);
}

void oracle_lattice(int *ex, int *ey, double *w, double *M, double *Minv)
{
    double inv[Q][Q];
    invert9(MM, inv);
    for (int i = 0; i < Q; ++i) {
        ex[i] = EX[i];
        ey[i] = EY[i];
        w[i] = WT[i];
        for (int j = 0; j < Q; ++j) {
            M[i * Q + j] = MM[i][j];
            Minv[i * Q + j] = inv[i][j];
        }
    }
}

void oracle_lattice5(double *M, double *Minv)
{
    double inv[Q5][Q5];
    invert5(M5, inv);
    for (int i = 0; i < Q5; ++i)
        for (int j = 0; j < Q5; ++j) {
            M[i * Q5 + j] = M5[i][j];
            Minv[i * Q5 + j] = inv[i][j];
        }
}

/* ------------------------------------------------------------------ */
/* Geometry helpers.                                                   */
/* ------------------------------------------------------------------ */
static int wall_of(const oracle_params *p, int X, int Y)
{
    if (!p->periodic_x) {
        if (X == 0) return W_LEFT; /* corners belong to the vertical walls */
        if (X == p->NX - 1) return W_RIGHT;
    }
    if (Y == 0) return W_BOTTOM;
    if (Y == p->NY - 1) return W_TOP;
    return W_NONE;
}

/* Wall whose thermal condition node (X, Y) carries: an isothermal vertical
 * wall, else an isothermal horizontal wall, else W_NONE (adiabatic). */
static int thermal_wall_of(const oracle_params *p, int X, int Y)
{
    int v = W_NONE, h = W_NONE;
    if (!p->periodic_x) {
        if (X == 0) v = W_LEFT;
        else if (X == p->NX - 1) v = W_RIGHT;
    }
    if (Y == 0) h = W_BOTTOM;
    else if (Y == p->NY - 1) h = W_TOP;
    if (v != W_NONE && p->wall_type[v] == WALL_ISOTHERMAL) return v;
    if (h != W_NONE && p->wall_type[h] == WALL_ISOTHERMAL) return h;
    return W_NONE;
}

static void partner_of(const oracle_params *p, int X, int Y, int *PX, int *PY)
{
    *PX = X;
    *PY = Y;
    if (!p->periodic_x) {
        if (X == 0) *PX = 1;
        else if (X == p->NX - 1) *PX = p->NX - 2;
    }
    if (Y == 0) *PY = 1;
    else if (Y == p->NY - 1) *PY = p->NY - 2;
}

static inline long idx(const oracle_params *p, int x, int y) { return (long)y * p->nx + x; }

static int full_window(const oracle_params *p)
{
    return p->gx0 == 0 && p->gy0 == 0 && p->nx == p->NX && p->ny == p->NY;
}

/* ------------------------------------------------------------------ */
/* State management.                                                   */
/* ------------------------------------------------------------------ */
oracle_state *oracle_new(const oracle_params *p)
{
    if (p->nx < 1 || p->ny < 1 || p->NX < 4 || p->NY < 4) return NULL;
    if (p->periodic_x && (p->gx0 != 0 || p->nx != p->NX)) return NULL;
    oracle_state *s = (oracle_state *)calloc(1, sizeof(oracle_state));
    if (!s) return NULL;
    s->p = *p;
    if (p->qt != Q && p->qt != Q5) {
        free(s);
        return NULL;
    }
    if (invert9(MM, s->Minv) != 0 || invert5(M5, s->M5inv) != 0) {
        free(s);
        return NULL;
    }
    long n = (long)p->nx * p->ny;
    s->f = (double *)calloc((size_t)n * Q, sizeof(double));
    s->g = (double *)calloc((size_t)n * Q, sizeof(double));
    s->h = (double *)calloc((size_t)n * Q, sizeof(double));
    s->fs = (double *)calloc((size_t)n * Q, sizeof(double));
    s->gs = (double *)calloc((size_t)n * Q, sizeof(double));
    s->hs = (double *)calloc((size_t)n * Q, sizeof(double));
    s->srf = (double *)calloc((size_t)n, sizeof(double));
    s->srm = (double *)calloc((size_t)n, sizeof(double));
    s->valid = (unsigned char *)calloc((size_t)n, 1);
    s->valid_new = (unsigned char *)calloc((size_t)n, 1);
    if (!s->f || !s->g || !s->h || !s->fs || !s->gs || !s->hs || !s->srf || !s->srm || !s->valid ||
        !s->valid_new) {
        free(s->f); free(s->g); free(s->h); free(s->fs); free(s->gs); free(s->hs);
        free(s->srf); free(s->srm); free(s->valid); free(s->valid_new);
        free(s);
        return NULL;
    }
    return s;
}

void oracle_free(oracle_state *s)
{
    if (!s) return;
    free(s->f); free(s->g); free(s->h); free(s->fs); free(s->gs); free(s->hs);
    free(s->srf); free(s->srm); free(s->valid); free(s->valid_new);
    free(s);
}

static void totals(const oracle_state *s, double *E, double *Mass);

/* Initial state: equilibria (Eqs. 27, 40, 49) at rest, at the given
 * temperatures; isothermal wall nodes take their wall temperature.  The
 * previous-step sources equal the current ones, so the time-derivative term
 * of Eqs. (36) and (47) vanishes at the first step. */
void oracle_set_initial(oracle_state *s, const double *T_f0, const double *T_m0)
{
    const oracle_params *p = &s->p;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            long k = idx(p, x, y);
            int X = x + p->gx0, Y = y + p->gy0;
            double Tf = T_f0[k], Tm = T_m0[k];
            int w = thermal_wall_of(p, X, Y);
            if (w != W_NONE) Tf = Tm = p->wall_T[w];
            double H = oracle_enthalpy_of_T(p, Tf);
            oracle_feq(p->rho_l, 0.0, 0.0, p->phi, &s->f[k * Q]);
            geq_of(p, H, Tf, 0.0, 0.0, &s->g[k * Q]);
            heq_of(p, Tm, &s->h[k * Q]);
            s->srf[k] = p->h_v * (Tm - Tf) / (p->phi * p->rho_l);
            s->srm[k] = p->h_v * (Tf - Tm) / ((1.0 - p->phi) * p->rho_m);
            s->valid[k] = 1;
        }
    s->step = 0;
    for (int w = 0; w < 4; ++w) s->flux_E[w] = s->flux_M[w] = 0.0;
    totals(s, &s->E0, &s->M0);
}

/* Wall values and non-equilibrium extrapolation, Eq. (52) and its thermal
 * analogues, for wall node k with interior partner kp. */
static void reconstruct_wall(oracle_state *s, int X, int Y, long k, long kp)
{
    const oracle_params *p = &s->p;
    double *fb = &s->f[k * Q], *gb = &s->g[k * Q], *hb = &s->h[k * Q];
    const double *fp = &s->f[kp * Q], *gp = &s->g[kp * Q], *hp = &s->h[kp * Q];
    macros mf;
    node_macros(p, fp, gp, hp, &mf);
    double Tb, Hb, Tmb;
    int wall = thermal_wall_of(p, X, Y);
    if (wall != W_NONE) {
        Tb = Tmb = p->wall_T[wall];
        Hb = oracle_enthalpy_of_T(p, Tb);
    } else { /* adiabatic: zero normal gradient */
        Tb = mf.T_f;
        Hb = mf.H;
        Tmb = mf.T_m;
    }
    double eqb[Q], eqf[Q];
    /* flow: wall velocity 0, density of the partner */
    oracle_feq(mf.rho, 0.0, 0.0, p->phi, eqb);
    oracle_feq(mf.rho, mf.ux, mf.uy, p->phi, eqf);
    for (int i = 0; i < Q; ++i) fb[i] = eqb[i] + (fp[i] - eqf[i]);
    geq_of(p, Hb, Tb, 0.0, 0.0, eqb);
    geq_of(p, mf.H, mf.T_f, mf.ux, mf.uy, eqf);
    for (int i = 0; i < p->qt; ++i) gb[i] = eqb[i] + (gp[i] - eqf[i]);
    heq_of(p, Tmb, eqb);
    heq_of(p, mf.T_m, eqf);
    for (int i = 0; i < p->qt; ++i) hb[i] = eqb[i] + (hp[i] - eqf[i]);
}

/* One time step. */
static void step_once(oracle_state *s)
{
    const oracle_params *p = &s->p;
    const int nx = p->nx, ny = p->ny;
    const double we = p->phi * p->rho_l, wm = (1.0 - p->phi) * p->rho_m;

    /* 1-4: collisions at every node (wall nodes included). */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long k = idx(p, x, y);
            double srf_new, srm_new;
            collide_node(p, (const double(*)[Q])s->Minv, (const double(*)[Q5])s->M5inv,
                         &s->f[k * Q], &s->g[k * Q], &s->h[k * Q], s->srf[k], s->srm[k],
                         &s->fs[k * Q], &s->gs[k * Q], &s->hs[k * Q], &srf_new, &srm_new);
            s->srf[k] = srf_new;
            s->srm[k] = srm_new;
        }

    /* Wall link fluxes of this step (whole-cavity runs only). */
    if (full_window(p)) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long k = idx(p, x, y);
                int w = wall_of(p, x, y);
                for (int i = 0; i < Q; ++i) {
                    int tx = x + EX[i], ty = y + EY[i];
                    if (p->periodic_x) tx = (tx + nx) % nx;
                    if (tx < 0 || tx >= nx || ty < 0 || ty >= ny) continue;
                    int wt = wall_of(p, tx, ty);
                    /* energy moves only along the thermal lattice's links */
                    double e = i < p->qt ? we * s->gs[k * Q + i] + wm * s->hs[k * Q + i] : 0.0;
                    if (w != W_NONE && wt == W_NONE) { /* wall -> interior */
                        s->flux_E[w] += e;
                        s->flux_M[w] += s->fs[k * Q + i];
                    } else if (w == W_NONE && wt != W_NONE) { /* interior -> wall */
                        s->flux_E[wt] -= e;
                        s->flux_M[wt] -= s->fs[k * Q + i];
                    }
                }
            }
    }

    /* 5: streaming, Eqs. (15), (33), (44) (pull form of the same map). */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long k = idx(p, x, y);
            int ok = s->valid[k];
            for (int i = 0; i < Q; ++i) {
                int sx = x - EX[i], sy = y - EY[i];
                if (p->periodic_x) sx = (sx + nx) % nx;
                if (sx < 0 || sx >= nx || sy < 0 || sy >= ny) {
                    ok = 0; /* nothing streams in from outside the window */
                    continue;
                }
                long ks = idx(p, sx, sy);
                s->f[k * Q + i] = s->fs[ks * Q + i];
                if (i < p->qt) {
                    s->g[k * Q + i] = s->gs[ks * Q + i];
                    s->h[k * Q + i] = s->hs[ks * Q + i];
                }
                ok = ok && s->valid[ks];
            }
            s->valid_new[k] = (unsigned char)ok;
        }

    /* 6: wall nodes, rebuilt from their partners' new populations. */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int X = x + p->gx0, Y = y + p->gy0;
            int w = wall_of(p, X, Y);
            if (w == W_NONE) continue;
            long k = idx(p, x, y);
            int PX, PY;
            partner_of(p, X, Y, &PX, &PY);
            int px = PX - p->gx0, py = PY - p->gy0;
            if (px < 0 || px >= nx || py < 0 || py >= ny) {
                s->valid_new[k] = 0;
                continue;
            }
            long kp = idx(p, px, py);
            reconstruct_wall(s, X, Y, k, kp);
            s->valid_new[k] = s->valid_new[kp];
        }
    unsigned char *t = s->valid;
    s->valid = s->valid_new;
    s->valid_new = t;
    s->step += 1;
}

void oracle_step(oracle_state *s, long n)
{
    for (long t = 0; t < n; ++t) step_once(s);
}

/* ------------------------------------------------------------------ */
/* Outputs.                                                            */
/* ------------------------------------------------------------------ */
void oracle_fields(const oracle_state *s, double *ux, double *uy, double *T_f, double *T_m,
                   double *f_l, double *rho, unsigned char *valid)
{
    const oracle_params *p = &s->p;
    long n = (long)p->nx * p->ny;
    for (long k = 0; k < n; ++k) {
        macros m;
        node_macros(p, &s->f[k * Q], &s->g[k * Q], &s->h[k * Q], &m);
        if (ux) ux[k] = m.ux;
        if (uy) uy[k] = m.uy;
        if (T_f) T_f[k] = m.T_f;
        if (T_m) T_m[k] = m.T_m;
        if (f_l) f_l[k] = m.f_l;
        if (rho) rho[k] = m.rho;
        if (valid) valid[k] = s->valid[k];
    }
}

void oracle_populations(const oracle_state *s, double *f, double *g, double *h, double *srf)
{
    const oracle_params *p = &s->p;
    long n = (long)p->nx * p->ny;
    if (f) memcpy(f, s->f, sizeof(double) * (size_t)n * Q);
    if (g) memcpy(g, s->g, sizeof(double) * (size_t)n * Q);
    if (h) memcpy(h, s->h, sizeof(double) * (size_t)n * Q);
    if (srf) memcpy(srf, s->srf, sizeof(double) * (size_t)n);
}

/* Energy phi rho_l H + (1-phi) rho_m c_pm T_m and mass rho summed over the
 * non-wall nodes. */
static void totals(const oracle_state *s, double *E, double *Mass)
{
    const oracle_params *p = &s->p;
    double e = 0.0, m = 0.0;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            if (wall_of(p, x + p->gx0, y + p->gy0) != W_NONE) continue;
            long k = idx(p, x, y);
            double sg = 0.0, sh = 0.0, sf = 0.0;
            for (int i = 0; i < p->qt; ++i) {
                sg += s->g[k * Q + i];
                sh += s->h[k * Q + i];
            }
            for (int i = 0; i < Q; ++i) sf += s->f[k * Q + i];
            e += p->phi * p->rho_l * sg + (1.0 - p->phi) * p->rho_m * sh;
            m += sf;
        }
    *E = e;
    *Mass = m;
}

void oracle_diagnostics(const oracle_state *s, oracle_diag *d)
{
    const oracle_params *p = &s->p;
    const int nx = p->nx, ny = p->ny;
    memset(d, 0, sizeof(*d));
    d->step = (double)s->step;
    d->Fo = (double)s->step * (p->k_f / (p->rho_l * p->c_pl)) / (p->L * p->L);
    double *Tf = (double *)malloc(sizeof(double) * (size_t)nx * ny);
    double *Tm = (double *)malloc(sizeof(double) * (size_t)nx * ny);
    double *fl = (double *)malloc(sizeof(double) * (size_t)nx * ny);
    double *ux = (double *)malloc(sizeof(double) * (size_t)nx * ny);
    double *uy = (double *)malloc(sizeof(double) * (size_t)nx * ny);
    oracle_fields(s, ux, uy, Tf, Tm, fl, NULL, NULL);
    double sum_fl = 0.0, n_int = 0.0, dmax = 0.0, umax = 0.0, nonfinite = 0.0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long k = idx(p, x, y);
            for (int i = 0; i < Q; ++i)
                if (!isfinite(s->f[k * Q + i]) || !isfinite(s->g[k * Q + i]) ||
                    !isfinite(s->h[k * Q + i])) {
                    nonfinite += 1.0;
                    break;
                }
            if (wall_of(p, x + p->gx0, y + p->gy0) != W_NONE) continue;
            sum_fl += fl[k];
            n_int += 1.0;
            double dT = fabs(Tf[k] - Tm[k]);
            if (dT > dmax) dmax = dT;
            double um = sqrt(ux[k] * ux[k] + uy[k] * uy[k]);
            if (um > umax) umax = um;
        }
    d->liquid_fraction = sum_fl / n_int;
    d->max_dT_LTNE = dmax;
    d->u_max = umax;
    d->nonfinite = nonfinite;

    double dT = p->T_hot - p->T_cold;
    double ke = p->phi * p->k_f + (1.0 - p->phi) * p->k_m;
    if (!p->periodic_x && full_window(p)) {
        /* Hot-wall and cold-wall Nusselt numbers from second-order one-sided
         * differences, averaged over the non-corner wall nodes. */
        double qh = 0.0, qh_pcm = 0.0, qc = 0.0;
        for (int y = 1; y <= ny - 2; ++y) {
            double dTf = (-3.0 * Tf[idx(p, 0, y)] + 4.0 * Tf[idx(p, 1, y)] - Tf[idx(p, 2, y)]) / 2.0;
            double dTm = (-3.0 * Tm[idx(p, 0, y)] + 4.0 * Tm[idx(p, 1, y)] - Tm[idx(p, 2, y)]) / 2.0;
            qh += p->phi * p->k_f * dTf + (1.0 - p->phi) * p->k_m * dTm;
            qh_pcm += dTf;
            double cTf = (3.0 * Tf[idx(p, nx - 1, y)] - 4.0 * Tf[idx(p, nx - 2, y)] + Tf[idx(p, nx - 3, y)]) / 2.0;
            double cTm = (3.0 * Tm[idx(p, nx - 1, y)] - 4.0 * Tm[idx(p, nx - 2, y)] + Tm[idx(p, nx - 3, y)]) / 2.0;
            qc += p->phi * p->k_f * cTf + (1.0 - p->phi) * p->k_m * cTm;
        }
        double nrow = (double)(ny - 2);
        d->Nu_hot = -(p->L / (ke * dT)) * (qh / nrow);
        d->Nu_hot_pcm = -(p->L / dT) * (qh_pcm / nrow);
        d->Nu_cold = -(p->L / (ke * dT)) * (qc / nrow);
        /* Melt front on the middle row: first crossing of f_l = 0.5 seen
         * from the hot wall, linearly interpolated. */
        int jm = ny / 2;
        double xf = 1.0;
        if (fl[idx(p, 0, jm)] < 0.5) xf = 0.0;
        else
            for (int i = 0; i + 1 < nx; ++i) {
                double a = fl[idx(p, i, jm)], b = fl[idx(p, i + 1, jm)];
                if (a >= 0.5 && b < 0.5) {
                    xf = (i + (a - 0.5) / (a - b)) / p->L;
                    break;
                }
            }
        d->x_front_mid = xf;
    }
    double E, Mass;
    totals(s, &E, &Mass);
    d->E_int = E;
    d->E_int0 = s->E0;
    d->M_int = Mass;
    d->M_int0 = s->M0;
    double sE = 0.0, sM = 0.0;
    for (int w = 0; w < 4; ++w) {
        d->flux_E[w] = s->flux_E[w];
        d->flux_M[w] = s->flux_M[w];
        sE += s->flux_E[w];
        sM += s->flux_M[w];
    }
    d->energy_residual = E - s->E0 - sE;
    d->mass_residual = Mass - s->M0 - sM;
    free(Tf); free(Tm); free(fl); free(ux); free(uy);
}

/* Planting hook for failure-detection tests: overwrite one population. */
void oracle_poke(oracle_state *s, long node, int field, int dir, double value)
{
    double *a = field == 0 ? s->f : field == 1 ? s->g : s->h;
    a[node * Q + dir] = value;
}

long oracle_step_count(const oracle_state *s) { return s->step; }
