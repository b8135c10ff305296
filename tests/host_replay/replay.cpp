// CPU replay of the library's step kernels, built from the same headers the
// GPU kernels use (per-node arithmetic, multi-step tile logic, tile shapes,
// mapping and storage plan) with a host compiler, for AddressSanitizer and
// bit-level checks that need no GPU.
//
// Mode "kstep": after one first (non-pulling) step, advances a cavity by
// `launches` launches of K steps each, once with the one-step update at
// every node (the one-step kernel's per-node path) and once by emulating
// the K-step kernel's workgroups tile by tile: every thread of the first
// update, then (K = 3) every thread's pulls of the middle update before
// any of its writes, then the last update.  The LDS arrays of each emulated
// workgroup are exactly as large as the kernel's and filled with NaN bit
// patterns first, so a read of a slot no update wrote turns the result into
// NaN; the LBM_HOST_CHECK bounds checks of the headers are active.  The two
// state buffers (populations, previous-step sources) and the wall tallies
// must agree bit for bit.  Prints "identical" or the first difference.
//
// Mode "fields": the one-step path only, then the macroscopic fields of
// every node (u_x, u_y, T_f, T_m, f_l, rho as doubles, [field][ny][nx]) to
// the given file, for comparison with the oracle.
//
// Input on stdin: "key value" lines (the lbm_params fields by name, with
// wall_type/wall_T as four values; precision f64|f32|f32h64|f16|bf16|
// f16split|bf16split; mode; K; shape (tile shape index); launches; steps;
// seed; out), then "end".
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_node.h"
#include "lbm_plan.h"
#include "lbm_tiles.h"

static thread_local char g_err[512] = "";

lbm_status fail(lbm_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

using namespace lbm;

namespace {

struct Job {
    lbm_params p;
    lbm_precision prec = LBM_F32;
    std::string mode = "kstep", out;
    int K = 3, launches = 2, steps = 10, shape = 0;
    uint64_t seed = 1;
};

bool read_job(Job &j) {
    std::memset(&j.p, 0, sizeof(j.p));
    j.p.F_phi = -1.0;
    char key[64];
    while (scanf("%63s", key) == 1) {
        std::string k = key;
        if (k == "end") return true;
        auto rd = [](double &v) { return scanf("%lf", &v) == 1; };
        auto ri = [](int32_t &v) { return scanf("%d", &v) == 1; };
        bool ok = true;
        lbm_params &p = j.p;
        if (k == "nx") ok = ri(p.nx);
        else if (k == "ny") ok = ri(p.ny);
        else if (k == "bc_x") ok = ri(p.bc_x);
        else if (k == "gravity_axis") ok = ri(p.gravity_axis);
        else if (k == "porosity") ok = rd(p.porosity);
        else if (k == "Ra") ok = rd(p.Ra);
        else if (k == "Pr") ok = rd(p.Pr);
        else if (k == "Da") ok = rd(p.Da);
        else if (k == "Ste") ok = rd(p.Ste);
        else if (k == "k_ratio") ok = rd(p.k_ratio);
        else if (k == "cap_ratio") ok = rd(p.cap_ratio);
        else if (k == "Nu_i") ok = rd(p.Nu_i);
        else if (k == "F_phi") ok = rd(p.F_phi);
        else if (k == "dp_over_L") ok = rd(p.dp_over_L);
        else if (k == "k_f") ok = rd(p.k_f);
        else if (k == "cf_ref") ok = rd(p.cf_ref);
        else if (k == "cm_ref") ok = rd(p.cm_ref);
        else if (k == "J") ok = rd(p.J);
        else if (k == "T_hot") ok = rd(p.T_hot);
        else if (k == "T_cold") ok = rd(p.T_cold);
        else if (k == "T_init") ok = rd(p.T_init);
        else if (k == "T_solidus") ok = rd(p.T_solidus);
        else if (k == "T_liquidus") ok = rd(p.T_liquidus);
        else if (k == "thermal_lattice") ok = ri(p.thermal_lattice);
        else if (k == "thermal_collision") ok = ri(p.thermal_collision);
        else if (k == "varpi") ok = rd(p.varpi);
        else if (k == "zeta_e") ok = rd(p.zeta_e);
        else if (k == "wall_type") ok = ri(p.wall_type[0]) && ri(p.wall_type[1]) && ri(p.wall_type[2]) && ri(p.wall_type[3]);
        else if (k == "wall_T") ok = rd(p.wall_T[0]) && rd(p.wall_T[1]) && rd(p.wall_T[2]) && rd(p.wall_T[3]);
        else if (k == "L_char") ok = rd(p.L_char);
        else if (k == "solid_treatment") ok = ri(p.solid_treatment);
        else if (k == "band_rows") ok = ri(p.band_rows);
        else if (k == "pcm_even_rates") ok = ri(p.pcm_even_rates);
        else if (k == "K") ok = scanf("%d", &j.K) == 1;
        else if (k == "shape") ok = scanf("%d", &j.shape) == 1;
        else if (k == "launches") ok = scanf("%d", &j.launches) == 1;
        else if (k == "steps") ok = scanf("%d", &j.steps) == 1;
        else if (k == "seed") ok = scanf("%llu", (unsigned long long *)&j.seed) == 1;
        else if (k == "mode" || k == "precision" || k == "out") {
            char v[512];
            ok = scanf("%511s", v) == 1;
            if (k == "mode") j.mode = v;
            else if (k == "out") j.out = v;
            else {
                const std::string s = v;
                if (s == "f64") j.prec = LBM_F64;
                else if (s == "f32") j.prec = LBM_F32;
                else if (s == "f32h64") j.prec = LBM_F32_H64;
                else if (s == "f16") j.prec = LBM_F16_OFFSET;
                else if (s == "bf16") j.prec = LBM_BF16_OFFSET;
                else if (s == "f16split") j.prec = LBM_F16_SPLIT;
                else if (s == "bf16split") j.prec = LBM_BF16_SPLIT;
                else ok = false;
            }
        } else {
            fprintf(stderr, "replay: unknown key %s\n", key);
            return false;
        }
        if (!ok) {
            fprintf(stderr, "replay: bad value for %s\n", key);
            return false;
        }
    }
    return false;
}

// One cavity's state in host memory, laid out as in the library's buffers.
template <int ST>
struct State {
    using Lay = typename LayoutOf<ST>::L;
    using R = typename LayoutOf<ST>::R;
    std::vector<unsigned char> pop[2];
    std::vector<R> sr[2];
    std::vector<double> acc;
};

// Deterministic perturbation of the interior PCM temperature (a 64-bit LCG).
double noise(uint64_t &s) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return ((double)(s >> 11) / 9007199254740992.0 - 0.5) * 2e-6;
}

template <int ST>
void one_step_all(const CavityConst<typename LayoutOf<ST>::R> &c, State<ST> &S, int cur, bool pull) {
    using Lay = typename LayoutOf<ST>::L;
    using R = typename LayoutOf<ST>::R;
    using RH = typename LayoutOf<ST>::RH;
    for (int y = 0; y < c.ny; ++y)
        for (int x = 0; x < c.nx; ++x) {
            if (pull)
                step_node<Lay, R, RH, true>(c, S.pop[cur].data(), S.pop[1 - cur].data(), S.sr[cur].data(),
                                            S.sr[1 - cur].data(), S.acc.data(), x, y);
            else
                step_node<Lay, R, RH, false>(c, S.pop[cur].data(), S.pop[1 - cur].data(), S.sr[cur].data(),
                                             S.sr[1 - cur].data(), S.acc.data(), x, y);
        }
}

// One K-step launch over every tile, each tile an emulated workgroup (tile
// shape I).
template <int ST, int K, int I>
void k_step_all(const CavityConst<typename LayoutOf<ST>::R> &c, State<ST> &S, int cur,
                const std::vector<Tile2> &tiles) {
    using Lay = typename LayoutOf<ST>::L;
    using R = typename LayoutOf<ST>::R;
    using RH = typename LayoutOf<ST>::RH;
    using Tl = StepKTileI<ST, K, I>;
    constexpr int TW = Tl::TW, TH = Tl::TH, NT = Tl::NT;
    using Sh = StepKShape<Lay, TW, TH, K>;
    static_assert(NT >= Sh::NFIRST, "one thread per node of the first update");
    for (const Tile2 &tl : tiles) {
        // LDS of the workgroup: exactly the kernel's sizes, NaN bit patterns
        std::vector<unsigned char> lds(Sh::LDS_BYTES, 0xff);
        std::vector<R> lds_sr(Sh::NSLOT);
        std::memset(lds_sr.data(), 0xff, lds_sr.size() * sizeof(R));
        std::vector<float> lds_b(Sh::STAGE_BASE ? 3 * Sh::NBASE : 1);
        std::memset(lds_b.data(), 0xff, lds_b.size() * sizeof(float));
        if constexpr (Sh::STAGE_BASE)
            for (int t = 0; t < NT; ++t)
                stepk_stage_bases<Lay, R, TW, TH, K, NT>(c, tl, S.pop[cur].data(), lds_b.data(), t);
        for (int s = 0; s < NT; ++s)
            if (s < Sh::LW * (tl.h + 2 * Sh::RING))
                stepk_first<Lay, R, RH, TW, TH, K>(c, tl, S.pop[cur].data(), S.sr[cur].data(), S.acc.data(),
                                                   lds.data(), lds_sr.data(), lds_b.data(), s);
        for (int j = K - 2; j >= 1; --j) {
            std::vector<MidNode<R, RH>> nodes(NT);
            std::vector<char> act(NT, 0);
            for (int t = 0; t < NT; ++t)
                act[t] = t < (TW + 2 * j) * (tl.h + 2 * j) &&
                         stepk_mid_load<Lay, R, RH, TW, TH, K>(c, tl, j, lds.data(), lds_sr.data(), t, nodes[t]);
            for (int t = 0; t < NT; ++t)
                if (act[t])
                    stepk_mid_store<Lay, R, RH, TW, TH, K>(c, tl, S.acc.data(), lds.data(), lds_sr.data(), nodes[t]);
        }
        for (int n = 0; n < NT; ++n)
            if (n < TW * tl.h)
                stepk_last<Lay, R, RH, TW, TH, K>(c, tl, S.pop[1 - cur].data(), S.sr[1 - cur].data(), S.acc.data(),
                                                  lds.data(), lds_sr.data(), n);
    }
}

template <int ST>
int run(const Job &j) {
    using Lay = typename LayoutOf<ST>::L;
    using R = typename LayoutOf<ST>::R;
    using RH = typename LayoutOf<ST>::RH;
    Lattice l;
    if (map_params(j.p, j.prec, l) != LBM_OK) {
        fprintf(stderr, "replay: %s\n", g_err);
        return 2;
    }
    const int nx = j.p.nx, ny = j.p.ny;
    const Bands bd = bands_of(nx, ny, Lay::bytes_per_node, 0, j.p.band_rows);
    const CavityConst<R> c = make_const<R>(l, 0, 0, bd);
    State<ST> S;
    const size_t pop_bytes = (size_t)bd.bytes * bd.count;
    const size_t nodes = (size_t)nx * ny;
    for (int b = 0; b < 2; ++b) {
        S.pop[b].assign(pop_bytes, 0);
        S.sr[b].assign(nodes, R(0));
    }
    S.acc.assign((size_t)4 * (nx + ny), 0.0);
    uint64_t s = j.seed;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double Tf = j.p.T_init;
            const bool interior = y > 0 && y < ny - 1 && (j.p.bc_x == 1 || (x > 0 && x < nx - 1));
            if (interior) Tf += noise(s);
            init_node<Lay, R, RH>(c, S.pop[0].data(), S.sr[0].data(), x, y, Tf, j.p.T_init);
        }
    if (j.mode == "fields") {
        // `steps` steps (the first one from the post-streaming initial state)
        int cur = 0;
        for (int t = 0; t < j.steps; ++t) {
            one_step_all<ST>(c, S, cur, t > 0);
            cur ^= 1;
        }
        std::vector<double> f((size_t)6 * nodes);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double out[6], v[NPART] = {0};
                macro_node<Lay, R, RH>(c, S.pop[cur].data(), j.steps == 0, x, y, out, v);
                for (int q = 0; q < 6; ++q) f[(size_t)q * nodes + (size_t)y * nx + x] = out[q];
            }
        FILE *fo = fopen(j.out.c_str(), "wb");
        if (!fo || fwrite(f.data(), sizeof(double), f.size(), fo) != f.size()) return 2;
        fclose(fo);
        printf("fields written\n");
        return 0;
    }
    // the first step: the initial state is post-streaming
    one_step_all<ST>(c, S, 0, false);
    int cur = 1;
    int tw = 0, th = 0;
    if (j.shape < 0 || j.shape >= kTileShapes) return 2;
    if constexpr (stepk_available(ST, 2)) {
        if (j.K == 2) {
            tw = dims_of<ST, 2>(j.shape).tw;
            th = dims_of<ST, 2>(j.shape).th;
        }
    }
    if constexpr (stepk_available(ST, 3)) {
        if (j.K == 3) {
            tw = dims_of<ST, 3>(j.shape).tw;
            th = dims_of<ST, 3>(j.shape).th;
        }
    }
    if (!tw) return 2;
    std::vector<Tile2> tiles;
    cavity_tiles2(0, nx, ny, tw, th, tiles);
    State<ST> A = S, B = S;
    int ca = cur, cb = cur;
    for (int launch = 0; launch < j.launches; ++launch) {
        for (int k = 0; k < j.K; ++k) {
            one_step_all<ST>(c, A, ca, true);
            ca ^= 1;
        }
        if constexpr (stepk_available(ST, 2)) {
            if (j.K == 2 && j.shape == 0) k_step_all<ST, 2, 0>(c, B, cb, tiles);
            if (j.K == 2 && j.shape == 1) k_step_all<ST, 2, 1>(c, B, cb, tiles);
            if (j.K == 2 && j.shape == 2) k_step_all<ST, 2, 2>(c, B, cb, tiles);
        }
        if constexpr (stepk_available(ST, 3)) {
            if (j.K == 3 && j.shape == 0) k_step_all<ST, 3, 0>(c, B, cb, tiles);
            if (j.K == 3 && j.shape == 1) k_step_all<ST, 3, 1>(c, B, cb, tiles);
            if (j.K == 3 && j.shape == 2) k_step_all<ST, 3, 2>(c, B, cb, tiles);
        }
        cb ^= 1;
    }
    // compare the live buffers (A advanced by K launches of one step swaps K
    // times, B once per launch)
    if (std::memcmp(A.pop[ca].data(), B.pop[cb].data(), pop_bytes) != 0) {
        size_t i = 0;
        while (A.pop[ca][i] == B.pop[cb][i]) ++i;
        printf("populations differ at byte %zu of %zu\n", i, pop_bytes);
        return 1;
    }
    if (std::memcmp(A.sr[ca].data(), B.sr[cb].data(), nodes * sizeof(R)) != 0) {
        printf("sources differ\n");
        return 1;
    }
    if (std::memcmp(A.acc.data(), B.acc.data(), A.acc.size() * sizeof(double)) != 0) {
        printf("wall tallies differ\n");
        return 1;
    }
    // the state moved and holds no NaN
    size_t nonfinite = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double out[6], v[NPART] = {0};
            macro_node<Lay, R, RH>(c, B.pop[cb].data(), false, x, y, out, v);
            if (v[P_NF] != 0.0) ++nonfinite;
        }
    if (nonfinite) {
        printf("%zu nodes hold non-finite populations\n", nonfinite);
        return 1;
    }
    printf("identical: %d launches of %d steps, %zu tiles of %dx%d, %d bands of %d rows\n", j.launches, j.K,
           tiles.size(), tw, th, bd.count, bd.rows);
    return 0;
}

}  // namespace

int main() {
    Job j;
    if (!read_job(j)) return 2;
    const int st = storage_of(j.prec, j.p.thermal_lattice == 5 ? 5 : 9);
    if (j.mode == "kstep" && !stepk_available(st, j.K)) {
        fprintf(stderr, "replay: storage %d has no %d-step kernel\n", st, j.K);
        return 2;
    }
    switch (st) {
        case ST_F64: return run<ST_F64>(j);
        case ST_F32: return run<ST_F32>(j);
        case ST_F16: return run<ST_F16>(j);
        case ST_BF16: return run<ST_BF16>(j);
        case ST_F16S: return run<ST_F16S>(j);
        case ST_BF16S: return run<ST_BF16S>(j);
        case ST_F32H: return run<ST_F32H>(j);
        case ST5_F64: return run<ST5_F64>(j);
        case ST5_F32: return run<ST5_F32>(j);
        case ST5_F32H: return run<ST5_F32H>(j);
    }
    fprintf(stderr, "replay: unknown storage\n");
    return 2;
}
