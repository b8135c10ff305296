// Three steps per launch by wavefront marching (tile shape kWaveShape),
// shared by the kernels and the CPU replay of the step kernels.
//
// A wavefront owns a strip of w <= 60 columns and h rows at (x0, y0).  Its
// 64 lanes hold columns x0 - 2 .. x0 + 61, one each, and it sweeps the
// strip bottom to top, one row per iteration: in iteration t, update j
// (j = 1, 2, 3) advances row t - (j - 1) over the strip grown by a ring of
// 3 - j nodes (two rows below and above the strip are the ring in y).
// Update 1 pulls from the global state (Eqs. 15, 33, 44).  Updates 2 and 3
// pull from the registers of the update before: a population of direction
// i is moved to the lane that pulls it (e_x = +-1: the neighbouring lane,
// a lane shift) as soon as it is produced and kept as long as a later row
// pulls it (e_y = -1: pulled at once by the row below; e_y = 0: one
// iteration later; e_y = +1: two iterations later).  Only the ring in x is
// advanced more than once per step, the wavefronts never wait for each
// other, and LDS holds only two rarely used stashes.
//
// A wall node pulls through its interior partner.  A lane on a vertical
// wall takes the pulled set of the neighbouring lane.  The bottom and top
// rows are advanced by updates 2 and 3 together with the row next to them,
// from that row's pulled set: row 0 with row 1 (its partner's pulls reach
// row 2, produced one iteration after row 1), row ny - 1 with row ny - 2
// (the next update pulls its e_y = -1 populations one iteration later,
// from the stash).  Populations are rounded to their stored form between
// updates (the LDS codecs), so a launch is bit-identical to three one-step
// launches, wall tallies included (each node of the strip tallies its own
// updates in step order).
#pragma once

#include "lbm_node.h"

namespace lbm {

constexpr int kWaveLanes = 64;
constexpr int kWaveCols = kWaveLanes - 4;  // strip columns per wavefront

// The populations (and Sr_f) a node hands to the next update.
template <typename R, typename RH>
struct WNode {
    R f[9], h[9];
    RH g[9];
    R sr;
};

// What update j + 1 still pulls from update j, for its next row p: the
// e_y = +1 populations of rows p - 1 (ua) and p (ub), the e_y = 0 ones of
// row p (ha), and Sr_f of row p (sa).  Only those directions are used.
template <typename R, typename RH>
struct WCarry {
    WNode<R, RH> ua, ha, ub;
    R sa;
};

// The registers of one lane kept from one iteration to the next ...
template <typename R, typename RH>
struct WLane {
    int lane;
    WCarry<R, RH> b[2];  // updates 1 -> 2 and 2 -> 3
};
// ... and those of one iteration: update 1's and 2's rows, a pulled set
// (a fresh set per iteration, so that no value of them is carried over).
template <typename R, typename RH>
struct WTemp {
    WNode<R, RH> o1, o2, p;
};

// Index of an e_y = -1 direction (4, 7, 8) among the three, and of an
// e_y = +1 direction (2, 5, 6).
__host__ __device__ constexpr int wave_dslot(int i) { return i == 4 ? 0 : (i == 7 ? 1 : 2); }
__host__ __device__ constexpr int wave_uslot(int i) { return i == 2 ? 0 : (i == 5 ? 1 : 2); }

// LDS stash of one wavefront, [..][lane]: a pulled set and its previous-
// step source (p), kept while the wall row next to its row is advanced;
// the e_y = +1 populations of row 0 of update 2 (read later in the same
// iteration) or the e_y = -1 ones of row ny - 1 of update 2 (read in the
// next iteration) (w; never both at once, as ny >= 4); Sr_f of row ny - 1
// of update 2 (szt) and of row 0 of updates 1 and 2 (sz).
template <typename R, typename RH>
struct WStash {
    struct P {
        R f[9][kWaveLanes], h[9][kWaveLanes], sr[kWaveLanes];
        RH g[9][kWaveLanes];
    };
    struct W {
        R f[3][kWaveLanes], h[3][kWaveLanes];
        RH g[3][kWaveLanes];
    };
    P p;
    W w;
    R szt[kWaveLanes], sz[2][kWaveLanes];
};

template <typename R>
struct WaveArgs {
    const CavityConst<R> *c;
    Tile2 tl;
    const void *src;
    void *dst;
    const R *sr_src;
    R *sr_dst;
    double *acc;
    bool left_wall, right_wall;  // the strip's lanes include a vertical wall
};

// Rows of update j in iteration t: row q; whether it is within the update's
// rows (lo <= q < hi, the strip grown by 3 - j rows, clipped to the cavity).
struct WRow {
    int q, lo, hi;
    bool act;
};
template <typename R>
LBM_HD WRow wave_row(const CavityConst<R> &c, const Tile2 &tl, int t, int j) {
    const int G = 3 - j;
    WRow r;
    r.q = t - (j - 1);
    r.lo = tl.y0 - G > 0 ? tl.y0 - G : 0;
    r.hi = tl.y0 + tl.h + G < c.ny ? tl.y0 + tl.h + G : c.ny;
    r.act = r.q >= r.lo && r.q < r.hi;
    return r;
}

// Column of a lane for an update with ring G: unwrapped x, wrapped xx, and
// whether the lane has a node.
template <typename R>
LBM_HD bool wave_col(const CavityConst<R> &c, const Tile2 &tl, int G, int lane, int &x, int &xx) {
    if (lane < 2 - G || lane >= 2 + tl.w + G) return false;
    x = tl.x0 - 2 + lane;
    xx = x;
    if (c.periodic) xx = x < 0 ? x + c.nx : (x >= c.nx ? x - c.nx : x);
    else if (x < 0 || x >= c.nx) return false;
    return true;
}

// A node's post-collision populations rounded to their stored form: what a
// one-step launch would load back (the LDS codec's encoding and decoding).
template <class Lay, typename R, typename RH>
LBM_HD void wave_round(const CavityConst<R> &c, R qf[9], RH qg[9], R qh[9], R bf, RH bg, R bh) {
    using Cd = LdsCodec<Lay>;
    alignas(16) unsigned char buf[Cd::bytes(1)];
    Cd::put_node(buf, 1, 0, c, qf, qg, qh, bf, bg, bh);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        qf[i] = Cd::template get<R>(buf, 1, 0, i, 0, c);
        if (i < Lay::QT) {
            qg[i] = Cd::template get<RH>(buf, 1, 1, i, 0, c);
            qh[i] = Cd::template get<R>(buf, 1, 2, i, 0, c);
        }
    }
}

// Update of the node at row y of a lane with ring G from its pulled set p
// (p.sr: the previous-step source).  LAST: writes the global state;
// otherwise out receives the rounded populations and Sr_f.
template <class Lay, typename R, typename RH, bool LAST, bool WALLS>
LBM_HD void wave_update(const WaveArgs<R> &a, int G, int lane, int y, WNode<R, RH> &p, WNode<R, RH> &out) {
    const CavityConst<R> &c = *a.c;
    const Tile2 &tl = a.tl;
    int x, xx;
    if (!wave_col(c, tl, G, lane, x, xx)) return;
    LBM_HOST_CHECK(y >= 0 && y < c.ny && xx >= 0 && xx < c.nx);
    const bool owned = x >= tl.x0 && x < tl.x0 + tl.w && y >= tl.y0 && y < tl.y0 + tl.h;
    const NodeGeom g = geometry<WALLS>(c, xx, y, true);
    Thermo<RH> th;
    Macro<R> m;
    const RH srf =
        update_node<Lay::QT, R, RH, true, WALLS>(c, g, xx, y, p.f, p.g, p.h, p.sr, owned, a.acc, th, m);
    const ThermalConst<RH> &t = thermal<RH>(c);
    if constexpr (LAST) {
        LBM_HOST_CHECK(x == xx);
        const NodeRef k = band_origin(c, y)(x, y);
        void *blk = band_block(c, a.dst, y / c.band_rows);
        const int64_t stride = c.band_nodes;
        Lay::template store<R>(blk, stride, 0, p.f, m.drho, k, c);
        Lay::template store<RH>(blk, stride, 1, p.g, t.c_fref * (th.Tf - t.T_ref), k, c);
        Lay::template store<R>(blk, stride, 2, p.h, c.c_mref * m.dTm, k, c);
        a.sr_dst[flat_index(c, x, y)] = (R)srf;
        (void)out;
    } else {
        wave_round<Lay, R, RH>(c, p.f, p.g, p.h, m.drho, t.c_fref * (th.Tf - t.T_ref), c.c_mref * m.dTm);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            out.f[i] = p.f[i];
            if (i < Lay::QT) {
                out.g[i] = p.g[i];
                out.h[i] = p.h[i];
            }
        }
        out.sr = (R)srf;
    }
}

// Update 1 of row y: pulls from the global state, then as wave_update.
template <class Lay, typename R, typename RH, bool WALLS>
LBM_HD void wave_first(const WaveArgs<R> &a, int lane, int y, WNode<R, RH> &p, WNode<R, RH> &out) {
    const CavityConst<R> &c = *a.c;
    int x, xx;
    if (!wave_col(c, a.tl, 2, lane, x, xx)) return;
    const NodeGeom g = geometry<WALLS>(c, xx, y, true);
    // the pulls reach rows g.sy - 1 .. g.sy + 1, within y - 2 .. y + 2 (a
    // first row the same for the whole wavefront)
    const int yb = y >= 2 ? y - 2 : 0;
    const BandOrigin org = band_origin(c, yb);
    LBM_HOST_CHECK(g.sy - 1 >= yb && g.sy + 1 < org.y_next + c.band_rows);
    gather_at<Lay, R, RH, true>(c, band_block(c, a.src, yb / c.band_rows), g, xx, y, org, p.f, p.g, p.h);
    p.sr = a.sr_src[flat_index(c, xx, y)];
    wave_update<Lay, R, RH, false, WALLS>(a, 2, lane, y, p, out);
}

// The pulled set of row p from a carry (rows p - 1 and p) and the e_y = -1
// populations of row p + 1 (dn).
template <int QT, typename R, typename RH>
LBM_HD void wave_pull(const WCarry<R, RH> &b, const WNode<R, RH> &dn, WNode<R, RH> &p) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ey = ey_of(i);
        const WNode<R, RH> &s = ey > 0 ? b.ua : (ey == 0 ? b.ha : dn);
        p.f[i] = s.f[i];
        if (i < QT) {
            p.g[i] = s.g[i];
            p.h[i] = s.h[i];
        }
    }
    p.sr = b.sa;
}

// The carry after the producing update advanced row q (o); `up` holds the
// e_y = +1 populations of row q - 1 (the carry's own ub, or those of the
// bottom row advanced together with row 1).
template <int QT, typename R, typename RH>
LBM_HD void wave_rotate(WCarry<R, RH> &b, const WNode<R, RH> &o, const WNode<R, RH> &up) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ey = ey_of(i);
        if (ey > 0) {
            b.ua.f[i] = up.f[i];
            b.ub.f[i] = o.f[i];
            if (i < QT) {
                b.ua.g[i] = up.g[i];
                b.ua.h[i] = up.h[i];
                b.ub.g[i] = o.g[i];
                b.ub.h[i] = o.h[i];
            }
        } else if (ey == 0) {
            b.ha.f[i] = o.f[i];
            if (i < QT) {
                b.ha.g[i] = o.g[i];
                b.ha.h[i] = o.h[i];
            }
        }
    }
    b.sa = o.sr;
}

template <int QT, typename R, typename RH>
LBM_HD void stash_put_p(WStash<R, RH> *s, int l, const WNode<R, RH> &p) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        s->p.f[i][l] = p.f[i];
        if (i < QT) {
            s->p.g[i][l] = p.g[i];
            s->p.h[i][l] = p.h[i];
        }
    }
    s->p.sr[l] = p.sr;
}
template <int QT, typename R, typename RH>
LBM_HD void stash_get_p(const WStash<R, RH> *s, int l, WNode<R, RH> &p) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        p.f[i] = s->p.f[i][l];
        if (i < QT) {
            p.g[i] = s->p.g[i][l];
            p.h[i] = s->p.h[i][l];
        }
    }
    p.sr = s->p.sr[l];
}
// The populations of o with e_y = EY (+1 or -1) into the stash, or from it
// into w.
template <int QT, int EY, typename R, typename RH>
LBM_HD void stash_put_w(WStash<R, RH> *s, int l, const WNode<R, RH> &o) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (ey_of(i) != EY) continue;
        const int k = EY > 0 ? wave_uslot(i) : wave_dslot(i);
        s->w.f[k][l] = o.f[i];
        if (i < QT) {
            s->w.g[k][l] = o.g[i];
            s->w.h[k][l] = o.h[i];
        }
    }
}
template <int QT, int EY, typename R, typename RH>
LBM_HD void stash_get_w(const WStash<R, RH> *s, int l, WNode<R, RH> &w) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (ey_of(i) != EY) continue;
        const int k = EY > 0 ? wave_uslot(i) : wave_dslot(i);
        w.f[i] = s->w.f[k][l];
        if (i < QT) {
            w.g[i] = s->w.g[k][l];
            w.h[i] = s->w.h[k][l];
        }
    }
}

// Lanes on a vertical wall take the pulled set of their partner's lane.
template <int QT, bool WALLS, class X, class T, typename R>
LBM_HD void wave_wall_fix(X &e, T &tmp, const WaveArgs<R> &a) {
    if constexpr (!WALLS) return;
    const int base = a.tl.x0 - 2, nx = a.c->nx;
    if (a.left_wall)
        e.template take<QT, -1>(tmp, [](auto &L, auto &M) -> auto & { return M.p; },
                                [=](const auto &L) { return base + L.lane == 0; });
    if (a.right_wall)
        e.template take<QT, +1>(tmp, [](auto &L, auto &M) -> auto & { return M.p; },
                                [=](const auto &L) { return base + L.lane == nx - 1; });
}

// One iteration of a wavefront's sweep.  X holds every lane's WLane, gives
// a fresh WTemp per lane (temps), runs a per-lane step on every lane
// (each), moves the populations of a node to the lanes that pull them
// (shift) and lets chosen lanes take the values of a neighbouring lane
// (take); st is the wavefront's stash.
template <class Lay, typename R, typename RH, bool WALLS, class X>
LBM_HD void wave_iteration(X &e, const WaveArgs<R> &a, WStash<R, RH> *st, int t) {
    constexpr int QT = Lay::QT;
    const CavityConst<R> &c = *a.c;
    const int ny = c.ny;
    const WRow s1 = wave_row(c, a.tl, t, 1), s2 = wave_row(c, a.tl, t, 2), s3 = wave_row(c, a.tl, t, 3);
    auto tmp = e.temps();
    auto O1 = [](auto &L, auto &M) -> auto & { return M.o1; };
    auto O2 = [](auto &L, auto &M) -> auto & { return M.o2; };

    // update 1, row s1.q
    if (s1.act) {
        e.each(tmp, [&](auto &L, auto &M) { wave_first<Lay, R, RH, WALLS>(a, L.lane, s1.q, M.p, M.o1); });
        e.template shift<QT>(tmp, O1);
        if (WALLS && s1.q == 0) e.each(tmp, [&](auto &L, auto &M) { st->sz[0][L.lane] = M.o1.sr; });
    }

    // update 2, row s2.q; rows 0 and ny - 1 go with rows 1 and ny - 2
    const bool u2 = s2.act && s2.q != 0 && s2.q != ny - 1;
    const bool bot2 = WALLS && u2 && s2.q == 1 && s2.lo == 0;
    const bool top2 = WALLS && u2 && s2.q == ny - 2 && ny - 1 < s2.hi;
    if (u2) {
        e.each(tmp, [&](auto &L, auto &M) { wave_pull<QT>(L.b[0], M.o1, M.p); });
        wave_wall_fix<QT, WALLS>(e, tmp, a);
        if (bot2 || top2) e.each(tmp, [&](auto &L, auto &M) { stash_put_p<QT>(st, L.lane, M.p); });
    }
    if (s1.act) e.each(tmp, [&](auto &L, auto &M) { wave_rotate<QT>(L.b[0], M.o1, L.b[0].ub); });
    if (u2) {
        if (bot2 || top2) {
            // the wall row first, from the same pulled set; what later rows
            // take from it goes to the stash
            e.each(tmp, [&](auto &L, auto &M) {
                M.p.sr = bot2 ? st->sz[0][L.lane] : M.o1.sr;  // Sr_f of row 0 / ny - 1 of update 1
                wave_update<Lay, R, RH, false, WALLS>(a, 1, L.lane, bot2 ? 0 : ny - 1, M.p, M.o2);
            });
            e.template shift<QT>(tmp, O2);
            e.each(tmp, [&](auto &L, auto &M) {
                stash_get_p<QT>(st, L.lane, M.p);
                if (bot2) {
                    stash_put_w<QT, +1>(st, L.lane, M.o2);
                    st->sz[1][L.lane] = M.o2.sr;
                } else {
                    stash_put_w<QT, -1>(st, L.lane, M.o2);
                    st->szt[L.lane] = M.o2.sr;
                }
            });
        }
        e.each(tmp, [&](auto &L, auto &M) { wave_update<Lay, R, RH, false, WALLS>(a, 1, L.lane, s2.q, M.p, M.o2); });
        e.template shift<QT>(tmp, O2);
    }

    // update 3, row s3.q, into the global state
    const bool u3 = s3.act && s3.q != 0 && s3.q != ny - 1;
    const bool bot3 = WALLS && u3 && s3.q == 1 && s3.lo == 0;
    const bool top3 = WALLS && u3 && s3.q == ny - 2 && ny - 1 < s3.hi;
    if (u3) {
        const bool early = WALLS && s2.q == ny - 1;  // update 2 advanced row ny - 1 an iteration ago
        e.each(tmp, [&](auto &L, auto &M) {
            if (early) {
                WNode<R, RH> dn;
                stash_get_w<QT, -1>(st, L.lane, dn);
                wave_pull<QT>(L.b[1], dn, M.p);
            } else {
                wave_pull<QT>(L.b[1], M.o2, M.p);
            }
        });
        wave_wall_fix<QT, WALLS>(e, tmp, a);
        if (bot3 || top3) e.each(tmp, [&](auto &L, auto &M) { stash_put_p<QT>(st, L.lane, M.p); });
    }
    if (u2) e.each(tmp, [&](auto &L, auto &M) {
        if (bot2) {  // row 0 of update 2, advanced with row 1, is the row before
            WNode<R, RH> up;
            stash_get_w<QT, +1>(st, L.lane, up);
            wave_rotate<QT>(L.b[1], M.o2, up);
        } else {
            wave_rotate<QT>(L.b[1], M.o2, L.b[1].ub);
        }
    });
    if (u3) {
        e.each(tmp, [&](auto &L, auto &M) { wave_update<Lay, R, RH, true, WALLS>(a, 0, L.lane, s3.q, M.p, M.p); });
        if (bot3 || top3) e.each(tmp, [&](auto &L, auto &M) {
            stash_get_p<QT>(st, L.lane, M.p);
            M.p.sr = bot3 ? st->sz[1][L.lane] : st->szt[L.lane];  // Sr_f of the wall row of update 2
            wave_update<Lay, R, RH, true, WALLS>(a, 0, L.lane, bot3 ? 0 : ny - 1, M.p, M.p);
        });
    }
}

// A wavefront's sweep of its strip, from update 1's first row to update
// 3's last; a strip whose updated nodes are all away from the walls takes
// the instantiation without the wall code.
template <class Lay, typename R, typename RH, class X>
LBM_HD void wave_sweep(X &e, const WaveArgs<R> &a, WStash<R, RH> *st) {
    const CavityConst<R> &c = *a.c;
    const Tile2 &tl = a.tl;
    const int t0 = wave_row(c, tl, 0, 1).lo, t1 = wave_row(c, tl, 0, 3).hi + 2;
    if (block_interior(c, tl.x0 - 2, tl.x0 + tl.w + 1, tl.y0 - 2, tl.y0 + tl.h + 1)) {
        for (int t = t0; t < t1; ++t) wave_iteration<Lay, R, RH, false>(e, a, st, t);
    } else {
        for (int t = t0; t < t1; ++t) wave_iteration<Lay, R, RH, true>(e, a, st, t);
    }
}

}  // namespace lbm
