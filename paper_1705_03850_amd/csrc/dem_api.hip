// dem_api.hip -- host side of libdem.so: validation, workspace layout, the
// step driver and the C-ABI declared in include/dem.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dem.h"
#include "dem_ctx.h"

using namespace dem;

namespace dem {
namespace host {

double cutoff_of(const dem_config &c) { return 2.0 * c.r_max + c.skin; }

bool material_ok(const dem_material &m) {
    return m.E > 0.0 && m.nu > -1.0 && m.nu < 0.5 && m.rho > 0.0 && m.e > 0.0 && m.e <= 1.0 && m.mu >= 0.0 &&
           std::isfinite(m.E) && std::isfinite(m.mu) && std::isfinite(m.rho);
}

// Eq. (6) with the effective properties of the two materials: harmonic E* and
// G*, arithmetic means of e and mu, folded into the per-contact factors.
PairCoef pair_coef(const dem_material &a, const dem_material &b) {
    double inv_E = (1.0 - a.nu * a.nu) / a.E + (1.0 - b.nu * b.nu) / b.E;
    double inv_G = 2.0 * (2.0 - a.nu) * (1.0 + a.nu) / a.E + 2.0 * (2.0 - b.nu) * (1.0 + b.nu) / b.E;
    double e = (a.e + b.e) / 2.0;
    double mu = (a.mu + b.mu) / 2.0;
    double le = std::log(e);
    const double Es = 1.0 / inv_E, Gs = 1.0 / inv_G;
    const double beta = le / std::sqrt(le * le + M_PI * M_PI);
    PairCoef k;
    memset(&k, 0, sizeof k);
    k.kn0 = 4.0 / 3.0 * Es;
    k.kt0 = 8.0 * Gs;
    k.gn0 = -beta * std::sqrt(20.0 / 3.0 * Es);
    k.gt0 = -beta * std::sqrt(80.0 / 3.0 * Gs);
    k.mu = mu;
    return k;
}

// Validates the configurations and derives the device descriptors.
int build_geometry(int32_t nsys, const dem_config *cfgs, Geometry &g, std::string &err) {
    if (nsys < 1 || !cfgs) { err = "need at least one system"; return DEM_ERR_ARG; }
    g = Geometry();
    g.block = cfgs[0].block == 0 ? 256 : cfgs[0].block;
    if (g.block != 64 && g.block != 128 && g.block != 256) { err = "block must be 64, 128 or 256"; return DEM_ERR_ARG; }
    for (int s = 0; s < nsys; ++s) {
        const dem_config &c = cfgs[s];
        char buf[256];
        if (c.ntypes < 1 || c.ntypes > DEM_MAX_TYPES) { err = "ntypes out of range"; return DEM_ERR_ARG; }
        for (int t = 0; t < c.ntypes; ++t) {
            const dem_material &m = c.mat[t];
            if (!material_ok(m)) {
                snprintf(buf, sizeof buf, "system %d type %d: need E > 0, -1 < nu < 0.5, rho > 0, 0 < e <= 1, mu >= 0", s, t);
                err = buf;
                return DEM_ERR_ARG;
            }
        }
        if (!(c.dt > 0.0) || !std::isfinite(c.dt)) { err = "dt must be > 0"; return DEM_ERR_ARG; }
        if (!(c.skin > 0.0)) { err = "skin must be > 0"; return DEM_ERR_ARG; }
        if (!(c.r_max > 0.0)) { err = "r_max must be > 0"; return DEM_ERR_ARG; }
        if (c.n < 0) { err = "n must be >= 0"; return DEM_ERR_ARG; }
        const int64_t slots = c.n_max == 0 ? c.n : c.n_max;
        if (slots < c.n) { err = "n_max must be 0 or >= n"; return DEM_ERR_ARG; }
        if (c.k_max < 1 || c.k_max > kMaxSlots) { err = "k_max must be in 1..63"; return DEM_ERR_ARG; }
        if (c.n_surf < 0 || c.n_surf > DEM_MAX_SURFACES) { err = "n_surf must be in 0..4"; return DEM_ERR_ARG; }
        if ((c.block == 0 ? 256 : c.block) != g.block) { err = "all systems of a batch need the same block size"; return DEM_ERR_ARG; }
        const double cut = cutoff_of(c);
        double h = c.cell > 0.0 ? c.cell : cut;
        if (h < cut) { err = "cell must be >= 2 r_max + skin"; return DEM_ERR_ARG; }
        SysDesc d;
        memset(&d, 0, sizeof d);
        int64_t cells = 1;
        for (int a = 0; a < 3; ++a) {
            if (!(c.hi[a] > c.lo[a])) { err = "box needs hi > lo"; return DEM_ERR_ARG; }
            d.lo[a] = c.lo[a];
            d.hi[a] = c.hi[a];
            d.L[a] = c.hi[a] - c.lo[a];
            d.hL[a] = 0.5 * d.L[a];
            d.periodic[a] = c.periodic[a] ? 1 : 0;
            d.g[a] = c.g[a];
            double want = d.L[a] / (h * (1.0 + 1e-9));
            int64_t nc = (int64_t)std::floor(want);
            if (nc < 1) nc = 1;
            if (d.periodic[a]) {
                if (d.L[a] < 2.0 * cut || nc < 2) {
                    snprintf(buf, sizeof buf, "system %d: periodic axis %d shorter than two cut-offs (or two cells)", s, a);
                    err = buf;
                    return DEM_ERR_DOMAIN;
                }
            }
            if (nc > (1 << 20)) { err = "too many cells along an axis"; return DEM_ERR_DOMAIN; }
            d.nc[a] = (int32_t)nc;
            d.inv_w[a] = (double)nc / d.L[a];
            cells *= nc;
        }
        d.dt = c.dt;
        d.hdt = 0.5 * c.dt;
        d.skin = c.skin;
        d.disp_thr2 = (0.5 * c.skin) * (0.5 * c.skin);
        d.rmax = c.r_max;
        d.p0 = g.n;
        d.p1 = g.n + slots;
        d.pe = g.n + c.n;
        d.c0 = g.ncell;
        d.wall = c.wall_z0 ? 1 : 0;
        d.stride = 1;
        d.nsurf = 0;
        d.surf0 = s * kMaxSurf;
        g.surf_cap.push_back(c.n_surf);
        g.nsurf_slots = std::max(g.nsurf_slots, c.n_surf);
        d.ntypes = c.ntypes;
        d.coef0 = (int32_t)g.coef.size();
        d.type0 = (int32_t)g.rho.size();
        for (int ti = 0; ti < c.ntypes; ++ti)
            for (int tj = 0; tj < c.ntypes; ++tj) g.coef.push_back(pair_coef(c.mat[ti], c.mat[tj]));
        for (int t = 0; t < c.ntypes; ++t) g.rho.push_back(c.mat[t].rho);
        for (int t = 0; t < c.ntypes; ++t) g.mat.push_back(c.mat[t]);
        g.sys.push_back(d);
        g.n += slots;
        g.ncell += cells + 1;   // the system's cells and its spare cell
        g.kmax = std::max(g.kmax, c.k_max);
    }
    if (g.n > INT32_MAX / 2 || g.ncell > INT32_MAX / 2) { err = "problem too large for 32-bit indices"; return DEM_ERR_ARG; }
    Surf none;
    memset(&none, 0, sizeof none);
    g.surf.assign(g.sys.size() * kMaxSurf, none);
    return DEM_OK;
}

Layout make_layout(const Geometry &g) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    const size_t n = (size_t)g.n, K = (size_t)g.kmax, C = (size_t)g.ncell;
    L.sys = take(g.sys.size() * sizeof(SysDesc));
    L.coef = take(g.coef.size() * sizeof(PairCoef));
    L.rho = take(g.rho.size() * sizeof(double));
    L.flags = take(sizeof(Flags));
    L.m = take(n * 8);
    L.inv_m = take(n * 8);
    L.inv_I = take(n * 8);
    L.disp = take(3 * n * 8);
    L.xiw = take(3 * n * 8);
    L.frame = take(n * 4);
    L.dead = take(n * 4);
    L.fext = take(3 * n * 8);
    for (int b = 0; b < 2; ++b) {
        L.nbr[b] = take(K * n * 4);
        L.cnt[b] = take(n * 4);
        L.xi[b] = take(K * n * sizeof(D4));
        L.mask[b] = take(n * 8);
        L.ids[b] = take(n * 4);
    }
    L.cell_of = take(n * 4);
    L.rank = take(n * 4);
    L.order = take(n * 4);
    L.cell_count = take((C + 1) * 4);
    L.cell_start = take((C + 1) * 4);
    L.scan_partial = take(((C + 1023) / 1024 + 1) * 4);
    L.shadow_d = take(kShadowD * n * 8);
    L.shadow_i = take(3 * n * 4);
    for (int b = 0; b < 2; ++b) {
        L.pos[b] = take(n * sizeof(D4));
        L.vel[b] = take(n * sizeof(D4));
        L.spin[b] = take(n * sizeof(D4));
    }
    L.im = take(n * sizeof(D2));
    L.sel = take(g.sys.size() * 4);
    L.lcur = take(g.sys.size() * 4);
    L.tile0 = take((g.sys.size() + 1) * 8);
    L.mtile0 = take((g.sys.size() + 1) * 8);
    L.msys = take(g.sys.size() * 4);
    L.mlevel = take(kMaxLevels * 8);
    L.surf = take(g.sys.size() * kMaxSurf * sizeof(Surf));
    L.sxi = L.smask = L.shadow_s = 0;
    if (g.nsurf_slots > 0) {
        const size_t S = (size_t)g.nsurf_slots;
        L.sxi = take(S * n * sizeof(D4));
        L.smask = take(n * 4);
        L.shadow_s = take(3 * S * n * 8 + n * 4);
    }
    L.total = o;
    return L;
}

// First tile of every system for the fused step at the current launch shape
// (tiles of block / lanes particles over each system's live particles, none
// shared by two systems); uploaded again when insertions or removals change
// the live counts.
int upload_tiles(dem_ctx *c) {
    const int64_t ppb = c->geo.block / c->lanes;
    std::vector<int64_t> t0(c->geo.sys.size() + 1, 0);
    for (size_t s = 0; s < c->geo.sys.size(); ++s) {
        const int64_t ns = c->geo.sys[s].pe - c->geo.sys[s].p0;
        t0[s + 1] = t0[s] + (ns + ppb - 1) / ppb;
    }
    c->ntiles_b = t0.back();
    // the same tiles in the order of the systems' strides (multi-rate stepping)
    const size_t ns = c->geo.sys.size();
    std::vector<int32_t> ms(ns);
    for (size_t k = 0; k < ns; ++k) ms[k] = (int32_t)k;
    std::stable_sort(ms.begin(), ms.end(),
                     [&](int32_t p, int32_t q) { return c->geo.sys[p].stride < c->geo.sys[q].stride; });
    std::vector<int64_t> mt(ns + 1, 0), lv(kMaxLevels, 0);
    for (size_t k = 0; k < ns; ++k) mt[k + 1] = mt[k] + (t0[ms[k] + 1] - t0[ms[k]]);
    for (int l = 0; l < kMaxLevels; ++l) {
        int64_t e = 0;
        for (size_t k = 0; k < ns; ++k)
            if (c->geo.sys[ms[k]].stride <= (1 << l)) e = mt[k + 1];
        lv[l] = e;
    }
    HIPCALL(c, hipMemcpyAsync(c->ws + c->lay.tile0, t0.data(), t0.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCALL(c, hipMemcpyAsync(c->ws + c->lay.mtile0, mt.data(), mt.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCALL(c, hipMemcpyAsync(c->ws + c->lay.msys, ms.data(), ms.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCALL(c, hipMemcpyAsync(c->ws + c->lay.mlevel, lv.data(), lv.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCALL(c, hipStreamSynchronize(c->stream));
    return DEM_OK;
}

int fail(dem_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(dem_ctx *c, hipError_t e, const char *what) {
    return fail(c, DEM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}


KArgs kargs(dem_ctx *c, const dem_state *s) {
    KArgs a;
    memset(&a, 0, sizeof a);
    a.x = s->x; a.v = s->v; a.w = s->w; a.f = s->f; a.t = s->t; a.r = s->r;
    a.type = s->type; a.id = s->id;
    char *w = c->ws;
    const Layout &L = c->lay;
    a.m = (double *)(w + L.m);
    a.inv_m = (double *)(w + L.inv_m);
    a.inv_I = (double *)(w + L.inv_I);
    a.disp = (double *)(w + L.disp);
    a.xiw = (double *)(w + L.xiw);
    a.frame = (int32_t *)(w + L.frame);
    a.dead = (int32_t *)(w + L.dead);
    a.fext_ws = (double *)(w + L.fext);
    a.fext = c->fext_on ? a.fext_ws : nullptr;
    a.sys = c->d_sys;
    a.coef = c->d_coef;
    a.rho = c->d_rho;
    a.nsys = (int32_t)c->geo.sys.size();
    a.kmax = c->geo.kmax;
    a.block = c->geo.block;
    // default: as many workgroups as stay resident (the step kernel runs 4
    // waves per SIMD, 16 per CU), each walking several tiles; the dispatch of
    // every extra workgroup costs time
    a.grid_cap = (int32_t)(c->grid_cap > 0 ? c->grid_cap : (int64_t)c->cus * 16 * 64 / c->geo.block);
    a.lanes = c->lanes;
    a.multirate = c->multirate ? 1 : 0;
    a.n = c->geo.n;
    a.ncell = c->geo.ncell;
    a.call_steps = 0;
    a.only_sys = -1;
    a.w0 = c->win_on ? c->win[0] : 0;
    a.w1 = c->win_on ? c->win[1] : c->geo.n;
    a.cw0 = c->win_on ? c->win[2] : 0;
    a.cw1 = c->win_on ? c->win[3] : c->geo.ncell;
    a.flags = c->d_flags;
    a.lst[0] = c->lists[0];
    a.lst[1] = c->lists[1];
    a.cell_of = (int32_t *)(w + L.cell_of);
    a.rank = (int32_t *)(w + L.rank);
    a.order = (int32_t *)(w + L.order);
    a.cell_count = (int32_t *)(w + L.cell_count);
    a.cell_start = (int32_t *)(w + L.cell_start);
    a.scan_partial = (int32_t *)(w + L.scan_partial);
    a.shadow_d = (double *)(w + L.shadow_d);
    a.shadow_i = (int32_t *)(w + L.shadow_i);
    for (int b = 0; b < 2; ++b) {
        a.pos[b] = (D4 *)(w + L.pos[b]);
        a.vel[b] = (D4 *)(w + L.vel[b]);
        a.spin[b] = (D4 *)(w + L.spin[b]);
    }
    a.im = (D2 *)(w + L.im);
    a.sel = (int32_t *)(w + L.sel);
    a.tile0 = (const int64_t *)(w + L.tile0);
    a.mtile0 = (const int64_t *)(w + L.mtile0);
    a.msys = (const int32_t *)(w + L.msys);
    a.mlevel = (const int64_t *)(w + L.mlevel);
    a.ntiles_b = c->ntiles_b;
    a.lcur = (int32_t *)(w + L.lcur);
    a.surf = (const Surf *)(w + L.surf);
    a.nsurf_slots = c->geo.nsurf_slots;
    if (c->geo.nsurf_slots > 0) {
        a.sxi = (D4 *)(w + L.sxi);
        a.smask = (uint32_t *)(w + L.smask);
        a.shadow_s = (double *)(w + L.shadow_s);
    }
    return a;
}

int check_state(dem_ctx *c, const dem_state *s) {
    if (!c) return DEM_ERR_ARG;
    if (!s) return fail(c, DEM_ERR_ARG, "state is NULL");
    if (c->geo.n > 0 && (!s->x || !s->v || !s->w || !s->f || !s->t || !s->r || !s->type || !s->id))
        return fail(c, DEM_ERR_ARG, "a state array is NULL");
    return DEM_OK;
}

int read_flags(dem_ctx *c, Flags &h) {
    if (c->h_flags) {
        // into pinned memory, ordered on the stream: one wait instead of a
        // wait and a staged copy
        HIPCALL(c, hipMemcpyAsync(c->h_flags, c->d_flags, sizeof(Flags), hipMemcpyDeviceToHost, c->stream));
        HIPCALL(c, hipStreamSynchronize(c->stream));
        h = *c->h_flags;
        return DEM_OK;
    }
    HIPCALL(c, hipStreamSynchronize(c->stream));
    HIPCALL(c, hipMemcpy(&h, c->d_flags, sizeof(Flags), hipMemcpyDeviceToHost));
    return DEM_OK;
}

int flag_error(dem_ctx *c, const Flags &h) {
    if (h.err & kErrNonFinite) return fail(c, DEM_ERR_NONFINITE, "non-finite position or velocity");
    if (h.err & kErrCapacity) {
        char buf[160];
        snprintf(buf, sizeof buf, "neighbour row of %d entries exceeds k_max = %d", h.max_row, c->geo.kmax);
        return fail(c, DEM_ERR_CAPACITY, buf);
    }
    if (h.err & kErrCellOverflow) return fail(c, DEM_ERR_CAPACITY, "a cell holds more than 64 particles");
    if (h.err & kErrBadInput) return fail(c, DEM_ERR_ARG, "a particle has a type out of range, a negative id or r <= 0");
    if (h.err & kErrStale)
        return fail(c, DEM_ERR_STATE,
                    "cell fields found a sphere more than one list cell from its binned position (the list did not "
                    "match the positions): step or rebuild first");
    return DEM_OK;
}

// all: rebuild every system; otherwise only those whose step flagged them
int do_bin(dem_ctx *c, const dem_state *s, bool all) {
    KArgs a = kargs(c, s);
    if (all || !c->have_list) HIPCALL(c, launch_fill_i32(a.sel, (int64_t)c->geo.sys.size(), 1, c->stream));
    HIPCALL(c, launch_bin(a, c->frame_identity ? 1 : 0, c->stream));
    c->binned = true;
    c->frame_identity = false;
    c->list_current = false;
    return DEM_OK;
}

int do_neighbors(dem_ctx *c, const dem_state *s, bool clear_sel) {
    if (!c->binned) return fail(c, DEM_ERR_STATE, "dem_neighbors needs dem_bin on the current positions");
    int have_old = c->have_list ? 1 : 0;
    KArgs a = kargs(c, s);
    // each selected system builds into its other buffer, then switches to it
    HIPCALL(c, launch_neighbors(a, have_old, c->stream));
    HIPCALL(c, launch_flip(a, c->stream));
    if (clear_sel) HIPCALL(c, launch_fill_i32(a.sel, (int64_t)c->geo.sys.size(), 0, c->stream));
    HIPCALL(c, launch_ctrl(c->d_flags, 4, 1, c->stream));
    c->have_list = true;
    c->list_current = true;
    c->frame_identity = true;
    return DEM_OK;
}

int live_list(dem_ctx *c, int sy, List &out) {
    int32_t cur = 0;
    HIPCALL(c, hipStreamSynchronize(c->stream));
    HIPCALL(c, hipMemcpy(&cur, c->ws + c->lay.lcur + 4 * (size_t)sy, 4, hipMemcpyDeviceToHost));
    out = c->lists[cur & 1];
    return DEM_OK;
}

// Event pair around the next launch(es) of class `kind` when timing is on.
int tic(dem_ctx *c, int kind) {
    if (!c->timing) return DEM_OK;
    if ((size_t)(2 * c->ev_used + 2) > c->ev.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            HIPCALL(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
        c->ev_kind.resize(c->ev.size() / 2);
        c->ev_count.resize(c->ev.size() / 2);
    }
    c->ev_kind[c->ev_used] = kind;
    HIPCALL(c, hipEventRecord(c->ev[2 * c->ev_used], c->stream));
    return DEM_OK;
}

// Closes the pair opened by tic; `launches` kernels of its class ran in between.
int toc(dem_ctx *c, int launches = 1) {
    if (!c->timing) return DEM_OK;
    HIPCALL(c, hipEventRecord(c->ev[2 * c->ev_used + 1], c->stream));
    c->ev_count[c->ev_used] = launches;
    ++c->ev_used;
    return DEM_OK;
}

// After a synchronisation: fold the recorded pairs into the totals.
int collect_times(dem_ctx *c) {
    for (int k = 0; k < c->ev_used; ++k) {
        float ms = 0.0f;
        HIPCALL(c, hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
        c->t_ms[c->ev_kind[k]] += ms;
        c->t_n[c->ev_kind[k]] += c->ev_count[k];
    }
    c->ev_used = 0;
    return DEM_OK;
}

// The particle and cell index ranges spanned by the systems that asked for a
// rebuild (read from the device after the group's synchronisation).
int set_rebuild_window(dem_ctx *c) {
    std::vector<int32_t> sel(c->geo.sys.size());
    HIPCALL(c, hipMemcpy(sel.data(), c->ws + c->lay.sel, sel.size() * 4, hipMemcpyDeviceToHost));
    int64_t w0 = INT64_MAX, w1 = 0, cw0 = INT64_MAX, cw1 = 0;
    for (size_t k = 0; k < sel.size(); ++k) {
        if (!sel[k]) continue;
        const SysDesc &d = c->geo.sys[k];
        const int64_t cells = (int64_t)d.nc[0] * d.nc[1] * d.nc[2] + 1;   // with the spare cell
        w0 = std::min(w0, d.p0);
        w1 = std::max(w1, d.p1);
        cw0 = std::min(cw0, d.c0);
        cw1 = std::max(cw1, d.c0 + cells);
    }
    if (w0 == INT64_MAX) return DEM_OK;   // nothing selected: full ranges
    c->win[0] = w0; c->win[1] = w1; c->win[2] = cw0; c->win[3] = cw1;
    c->win_on = true;
    return DEM_OK;
}

// One graph of `len` fused steps starting from packed buffer 0 (k = 0..len-1).
int capture_graph(dem_ctx *c, const dem_state *s, GraphSlot &gs, int len) {
    if (gs.exec) { (void)hipGraphExecDestroy(gs.exec); gs.exec = nullptr; }
    KArgs a = kargs(c, s);
    hipGraph_t graph = nullptr;
    HIPCALL(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < len && e == hipSuccess; ++k)
        e = launch_step(a, k & 1, 1, k, 1, c->count ? 1 : 0, c->stream);
    hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch during graph capture");
    if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
    hipError_t e3 = hipGraphInstantiate(&gs.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) { gs.exec = nullptr; return hip_fail(c, e3, "hipGraphInstantiate"); }
    const void *key[10] = {c->ws, c->fext_on ? (const void *)c->lay.fext : nullptr,
                             c->multirate ? (const void *)c->lay.sys : nullptr};
    memcpy(gs.key, key, sizeof key);
    gs.chunk = len;
    gs.count = c->count ? 1 : 0;
    return DEM_OK;
}

// Running estimate of the steps between rebuilds (it sets the group length).
void note_rebuild(dem_ctx *c, int64_t ran) {
    const double gap = (double)(c->since_rebuild + ran);
    c->gap_avg = 0.5 * (c->gap_avg < 1e8 ? c->gap_avg : gap) + 0.5 * gap;
    c->since_rebuild = 0;
}

void note_steps(dem_ctx *c, int64_t ran) {
    c->since_rebuild += ran;
    if ((double)c->since_rebuild > c->gap_avg) c->gap_avg = (double)c->since_rebuild;
}

// The drift into step qa (1-based within the current call) asked for a new
// list: the systems that asked for it are unpacked, rebuilt and repacked into
// the same buffer, by kernels over the index window of those systems.
int rebuild_at(dem_ctx *c, const dem_state *s, int64_t qa) {
    const int buf = (int)((qa - 1) & 1);
    int rc;
    if ((rc = tic(c, 3))) return rc;
    if (c->geo.sys.size() > 1 && (rc = set_rebuild_window(c))) return rc;
    KArgs a = kargs(c, s);
    HIPCALL(c, launch_unpack(a, buf, 1, c->stream, qa));
    c->binned = false;
    if ((rc = do_bin(c, s, false)) || (rc = do_neighbors(c, s, false))) return rc;
    KArgs b = kargs(c, s);
    HIPCALL(c, launch_pack(b, buf, 2, 0, 0, c->stream, qa));
    c->win_on = false;
    HIPCALL(c, launch_fill_i32(b.sel, (int64_t)c->geo.sys.size(), 0, c->stream));
    return toc(c);
}

// Steps q..nsteps of a call whose first step is global step base + 1.  On
// entry the state of step q after its drift is in packed buffer (q - 1) & 1
// and the flag block's step base is base + q.  Steps are numbered
// 1..nsteps; the fused kernel of step q computes its forces and kicks, then
// drifts into q + 1.  Groups of launches run between synchronisations; a
// group that needs a rebuild stops at the step whose drift asked for it.
// The call's last step writes the caller's arrays.  h: the flags read after
// the last group.
int step_loop(dem_ctx *c, const dem_state *s, int64_t nsteps, int64_t base, int64_t q, Flags &h) {
    int rc;
    const int cnt = c->count ? 1 : 0;
    int64_t q0 = q;
    while (q <= nsteps) {
        KArgs a = kargs(c, s);
        // group length: the full chunk, or shorter while rebuilds come often (a
        // rebuild stops the group; the rest of it would run as empty launches)
        int len = c->chunk;
        if (c->gap_avg < 2.0 * c->chunk) {
            len = 8;
            while (2 * len <= c->chunk && 2 * len <= c->gap_avg / 2) len *= 2;
            if (len > c->chunk) len = c->chunk;
        }
        int slot = 0;
        while ((8 << slot) < len && slot < 7) ++slot;
        int pair1 = -1, pair2 = -1;   // timed event pairs of this group (fused steps, last step)
        if (c->use_graph && !c->timing && (8 << slot) == len && q == q0 && ((q - 1) & 1) == 0 &&
            q + len - 1 <= nsteps - 1) {
            GraphSlot &gs = c->graphs[slot];
            const void *key[10] = {c->ws, c->fext_on ? (const void *)c->lay.fext : nullptr,
                             c->multirate ? (const void *)c->lay.sys : nullptr};
            if (!gs.exec || memcmp(gs.key, key, sizeof key) || gs.chunk != len || gs.count != cnt)
                if ((rc = capture_graph(c, s, gs, len))) return rc;
            HIPCALL(c, hipGraphLaunch(gs.exec, c->stream));
            q += len;
        } else {
            // with timing on, one pair of events brackets each run of fused
            // steps (the last step of a call gets a pair of its own), so the
            // events add no gaps between the kernels they time
            int open = 0;
            while (q <= nsteps && q - q0 < len) {
                const int last = q == nsteps;
                if (last && open) {
                    if ((rc = toc(c, open))) return rc;
                    open = 0;
                }
                if (last) {
                    pair2 = c->ev_used;
                    if ((rc = tic(c, 2))) return rc;
                } else if (!open) {
                    pair1 = c->ev_used;
                    if ((rc = tic(c, 1))) return rc;
                }
                KArgs al = a;
                if (last) al.call_steps = nsteps;
                HIPCALL(c, launch_step(al, (int)((q - 1) & 1), last ? 2 : 1, (int)(q - q0), 1, cnt, c->stream));
                if (last) {
                    if ((rc = toc(c))) return rc;
                } else {
                    ++open;
                }
                ++q;
            }
            if (open && (rc = toc(c, open))) return rc;
        }
        if ((rc = read_flags(c, h))) return rc;
        if (c->timing && h.abort_at != INT64_MAX) {
            // launches at or after the rebuild request did no work: count only
            // the fused steps that ran (their near-empty launches stay inside
            // the timed interval, a few microseconds each)
            const int64_t ran = h.abort_at - base - q0;
            if (pair1 >= 0 && c->ev_count[pair1] > ran) c->ev_count[pair1] = (int)(ran > 0 ? ran : 0);
            if (pair2 >= 0 && h.abort_at - base <= nsteps) c->ev_count[pair2] = 0;
        }
        if ((rc = collect_times(c))) return rc;
        if ((rc = flag_error(c, h))) return rc;
        if (h.abort_at != INT64_MAX) {
            // the drift into step q_a asked for a new list: rebuild on the caller's
            // arrays and repack into the same buffer
            const int64_t qa = h.abort_at - base;
            if ((rc = rebuild_at(c, s, qa))) return rc;
            note_rebuild(c, qa - q0);
            q = qa;
        } else {
            note_steps(c, q - q0);
        }
        if (q <= nsteps) {
            HIPCALL(c, launch_ctrl(c->d_flags, 0, base + q, c->stream));
            q0 = q;
        }
    }
    return DEM_OK;
}

}  // namespace host
}  // namespace dem

using namespace dem::host;

extern "C" {

int dem_batch_workspace_size(int32_t nsys, const dem_config *cfgs, size_t *bytes) {
    if (!bytes) return DEM_ERR_ARG;
    Geometry g;
    std::string err;
    int rc = build_geometry(nsys, cfgs, g, err);
    if (rc) return rc;
    *bytes = make_layout(g).total;
    return DEM_OK;
}

int dem_workspace_size(const dem_config *cfg, size_t *bytes) { return dem_batch_workspace_size(1, cfg, bytes); }

static std::string g_init_error;

// Default lanes per particle: the most of 4, 8 and 16 that keep the force pass
// within 65,536 threads (one wave per SIMD of the device), else 4.  Small
// systems cannot fill the device, and more lanes shorten each particle's chain
// of dependent loads: 2,000 spheres step in 9.0 us with 16 lanes against 13.5
// with 4, 5,154 in 11.9 us with 8 against 14.0; from about 17,000 particles 4
// lanes are fastest.
static int32_t default_lanes(int64_t n, int32_t block) {
    int32_t lanes = 4;
    for (int32_t l = 16; l > 4; l /= 2)
        if (l <= block && n * l <= 65536) { lanes = l; break; }
    return lanes;
}

}  // extern "C"

// A context on the given workspace; with pin_flags also a pinned host copy of
// the flag block (the static-workspace context allocates nothing).
static int init_ctx(dem_ctx **out, int32_t nsys, const dem_config *cfgs, void *workspace, size_t ws_bytes,
                    void *stream, bool pin_flags) {
    if (!out) return DEM_ERR_ARG;
    *out = nullptr;
    Geometry g;
    std::string err;
    int rc = build_geometry(nsys, cfgs, g, err);
    if (rc) { g_init_error = err; return rc; }
    Layout lay = make_layout(g);
    if (!workspace || ws_bytes < lay.total) { g_init_error = "workspace too small"; return DEM_ERR_ARG; }
    if ((uintptr_t)workspace % kAlign) { g_init_error = "workspace must be 256-byte aligned"; return DEM_ERR_ARG; }
    dem_ctx *c = new dem_ctx();
    c->geo = g;
    c->lay = lay;
    c->ws = (char *)workspace;
    c->stream = (hipStream_t)stream;
    c->d_sys = (SysDesc *)(c->ws + lay.sys);
    c->d_coef = (PairCoef *)(c->ws + lay.coef);
    c->d_rho = (double *)(c->ws + lay.rho);
    c->d_flags = (Flags *)(c->ws + lay.flags);
    c->lanes = default_lanes(g.n, g.block);
    if (pin_flags && hipHostMalloc((void **)&c->h_flags, sizeof(Flags), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        c->h_flags = nullptr;
    }
    for (int b = 0; b < 2; ++b) {
        c->lists[b].nbr = (int32_t *)(c->ws + lay.nbr[b]);
        c->lists[b].cnt = (int32_t *)(c->ws + lay.cnt[b]);
        c->lists[b].xi = (D4 *)(c->ws + lay.xi[b]);
        c->lists[b].mask = (uint64_t *)(c->ws + lay.mask[b]);
        c->lists[b].ids = (int32_t *)(c->ws + lay.ids[b]);
    }
    hipError_t e = hipMemcpyAsync(c->d_sys, g.sys.data(), g.sys.size() * sizeof(SysDesc), hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_coef, g.coef.data(), g.coef.size() * sizeof(PairCoef), hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_rho, g.rho.data(), g.rho.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + lay.surf, g.surf.data(), g.surf.size() * sizeof(Surf), hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess) e = launch_ctrl(c->d_flags, 2, 0, c->stream);
    if (e == hipSuccess && upload_tiles(c) != DEM_OK) e = hipErrorUnknown;
    if (e == hipSuccess) {
        int dev = 0, cus = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess && cus > 0) c->cus = cus;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        g_init_error = std::string("HIP error during init: ") + hipGetErrorString(e);
        if (c->h_flags) (void)hipHostFree(c->h_flags);
        delete c;
        return DEM_ERR_HIP;
    }
    *out = c;
    return DEM_OK;
}

extern "C" {

int dem_batch_init(dem_ctx **out, int32_t nsys, const dem_config *cfgs, void *workspace, size_t ws_bytes,
                   void *stream) {
    return init_ctx(out, nsys, cfgs, workspace, ws_bytes, stream, true);
}

int dem_init(dem_ctx **ctx, const dem_config *cfg, void *workspace, size_t ws_bytes, void *stream) {
    return dem_batch_init(ctx, 1, cfg, workspace, ws_bytes, stream);
}

}  // extern "C"

// ------------------------------------------------- static workspace (no allocation)
//
// dem_init_noalloc places a context's workspace in this array instead of a
// caller buffer.  Each device holds its own copy for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in).  One
// context per device may use it at a time.
static constexpr size_t kStaticWsBytes = (size_t)64 << 20;

static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices];          // device address of `scratch` on each device
const dem_ctx *g_static_owner[kMaxDevices];  // the context that uses it, if any

}  // namespace

extern "C" {

int dem_init_noalloc(dem_ctx **out, const dem_config *cfg, void *stream) {
    if (!out) return DEM_ERR_ARG;
    *out = nullptr;
    Geometry g;
    std::string err;
    int rc = build_geometry(1, cfg, g, err);
    if (rc) { g_init_error = err; return rc; }
    const size_t need = make_layout(g).total;
    if (need > kStaticWsBytes) {
        char buf[200];
        snprintf(buf, sizeof buf, "this system needs %zu bytes of workspace; the static workspace holds %zu (use dem_init)",
                 need, kStaticWsBytes);
        g_init_error = buf;
        return DEM_ERR_CAPACITY;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { g_init_error = std::string("hipGetDevice: ") + hipGetErrorString(e); return DEM_ERR_HIP; }
    if (dev < 0 || dev >= kMaxDevices) { g_init_error = "device index out of range"; return DEM_ERR_ARG; }
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_init_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return DEM_ERR_HIP;
        }
        g_static_ptr[dev] = p;
    }
    if (g_static_owner[dev]) {
        g_init_error = "the static workspace of this device is used by another context (dem_destroy it first)";
        return DEM_ERR_STATE;
    }
    // the array keeps the last context's contents: start from zeros
    e = launch_fill_u64((uint64_t *)g_static_ptr[dev], (int64_t)(need / 8), 0, (hipStream_t)stream);
    if (e != hipSuccess) { g_init_error = std::string("clearing the static workspace: ") + hipGetErrorString(e); return DEM_ERR_HIP; }
    rc = init_ctx(out, 1, cfg, g_static_ptr[dev], kStaticWsBytes, stream, false);
    if (rc) return rc;
    (*out)->static_dev = dev;
    g_static_owner[dev] = *out;
    return DEM_OK;
}

int dem_reset(dem_ctx *c, const dem_state *s) {
    int rc = check_state(c, s);
    if (rc) return rc;
    KArgs a = kargs(c, s);
    HIPCALL(c, launch_init_mass(a, c->stream));
    HIPCALL(c, launch_fill_f64(a.disp, 3 * c->geo.n, 0.0, c->stream));
    HIPCALL(c, launch_fill_f64(a.xiw, 3 * c->geo.n, 0.0, c->stream));
    HIPCALL(c, launch_fill_i32(a.dead, c->geo.n, 0, c->stream));
    if (a.smask) HIPCALL(c, launch_fill_i32((int32_t *)a.smask, c->geo.n, 0, c->stream));
    HIPCALL(c, launch_fill_i32(a.sel, (int64_t)c->geo.sys.size(), 0, c->stream));
    HIPCALL(c, launch_fill_i32(a.lcur, (int64_t)c->geo.sys.size(), 0, c->stream));
    Flags h;
    if ((rc = read_flags(c, h))) return rc;
    if ((rc = flag_error(c, h))) return rc;
    c->masses = true;
    c->have_list = false;
    c->list_current = false;
    c->binned = false;
    c->frame_identity = true;
    c->forces_valid = false;
    c->fext_on = false;
    return DEM_OK;
}

int dem_bin(dem_ctx *c, const dem_state *s) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!c->masses) return fail(c, DEM_ERR_STATE, "dem_reset first");
    return do_bin(c, s, true);
}

int dem_neighbors(dem_ctx *c, const dem_state *s) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!c->masses) return fail(c, DEM_ERR_STATE, "dem_reset first");
    return do_neighbors(c, s);
}

int dem_forces(dem_ctx *c, const dem_state *s, int update_history) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!c->list_current) return fail(c, DEM_ERR_STATE, "dem_forces needs a neighbour list for the current order");
    KArgs a = kargs(c, s);
    HIPCALL(c, launch_pack(a, 0, 0, 0, 0, c->stream));
    HIPCALL(c, launch_step(a, 0, 0, 0, update_history ? 1 : 0, 0, c->stream));
    c->forces_valid = true;
    return DEM_OK;
}

int dem_integrate(dem_ctx *c, const dem_state *s, int phase) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (phase != 0 && phase != 1) return fail(c, DEM_ERR_ARG, "phase must be 0 or 1");
    if (!c->masses) return fail(c, DEM_ERR_STATE, "dem_reset first");
    KArgs a = kargs(c, s);
    HIPCALL(c, launch_phase(a, phase, 0, 0, c->stream));
    if (phase == 0) {
        c->binned = false;
        c->forces_valid = false;
    }
    return DEM_OK;
}

int dem_declare_forces(dem_ctx *c) {
    if (!c) return DEM_ERR_ARG;
    c->forces_valid = true;
    return DEM_OK;
}

}  // extern "C"

namespace {

__global__ void k_clear_surface_bits(uint32_t *smask, int64_t p0, int64_t p1, uint32_t bits) {
    for (int64_t i = p0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p1; i += (int64_t)gridDim.x * blockDim.x)
        smask[i] &= ~bits;
}

}  // namespace

extern "C" {

int dem_set_surfaces(dem_ctx *c, int32_t sys, int32_t count, const dem_surface *surf) {
    if (!c) return DEM_ERR_ARG;
    if (sys < 0 || sys >= (int32_t)c->geo.sys.size()) return fail(c, DEM_ERR_ARG, "sys out of range");
    if (count < 0 || count > c->geo.surf_cap[sys])
        return fail(c, DEM_ERR_ARG, "count exceeds the surfaces reserved for the system (dem_config.n_surf)");
    if (count > 0 && !surf) return fail(c, DEM_ERR_ARG, "surf is NULL");
    Surf next[kMaxSurf];
    memset(next, 0, sizeof next);
    for (int k = 0; k < count; ++k) {
        const dem_surface &q = surf[k];
        const bool finite = std::isfinite(q.axis[0]) && std::isfinite(q.axis[1]) && std::isfinite(q.z0) &&
                            std::isfinite(q.z1) && std::isfinite(q.r0) && std::isfinite(q.r1);
        bool ok = finite && std::isfinite(q.mu) && q.kind >= DEM_SURF_CYLINDER && q.kind <= DEM_SURF_RING &&
                  q.r0 > 0.0;
        if (q.kind == DEM_SURF_CYLINDER || q.kind == DEM_SURF_CONE) ok = ok && q.z1 > q.z0;
        if (q.kind == DEM_SURF_CONE) ok = ok && q.r1 > 0.0;
        if (!ok) return fail(c, DEM_ERR_ARG, "bad surface record (kind, finite values, r0 > 0, z1 > z0, cone r1 > 0)");
        Surf &w = next[k];
        w.kind = q.kind;
        w.enabled = q.enabled ? 1 : 0;
        w.cx = q.axis[0];
        w.cy = q.axis[1];
        w.z0 = q.z0;
        w.z1 = q.z1;
        w.r0 = q.r0;
        w.r1 = q.r1;
        w.mu = q.mu;
        if (q.kind == DEM_SURF_CONE) {
            // unit generator from (r0, z0) to (r1, z1) and the inward unit normal of the section
            const double sr = q.r1 - q.r0, sz = q.z1 - q.z0, len = std::sqrt(sr * sr + sz * sz);
            w.len = len;
            w.ur = sr / len;
            w.uz = sz / len;
            w.mr = -sz / len;
            w.mz = sr / len;
        }
    }
    Surf *cur = &c->geo.surf[(size_t)sys * kMaxSurf];
    uint32_t changed = 0;
    for (int k = 0; k < kMaxSurf; ++k)
        if (memcmp(&cur[k], &next[k], sizeof(Surf)) != 0) changed |= 1u << k;
    memcpy(cur, next, sizeof next);
    SysDesc &d = c->geo.sys[sys];
    d.nsurf = count;
    HIPCALL(c, hipMemcpyAsync(c->ws + c->lay.surf + (size_t)sys * kMaxSurf * sizeof(Surf), cur, sizeof next,
                              hipMemcpyHostToDevice, c->stream));
    HIPCALL(c, hipMemcpyAsync(c->d_sys + sys, &d, sizeof(SysDesc), hipMemcpyHostToDevice, c->stream));
    if (changed && c->lay.smask && d.p1 > d.p0) {
        int64_t blocks = (d.p1 - d.p0 + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        k_clear_surface_bits<<<(int)blocks, 256, 0, c->stream>>>((uint32_t *)(c->ws + c->lay.smask), d.p0, d.p1,
                                                                 changed);
        HIPCALL(c, hipGetLastError());
    }
    HIPCALL(c, hipStreamSynchronize(c->stream));   // the host records above are copied from
    return DEM_OK;
}

int dem_set_multirate(dem_ctx *c, int enable) {
    if (!c) return DEM_ERR_ARG;
    std::vector<int32_t> stride(c->geo.sys.size(), 1);
    int32_t mx = 1;
    if (enable) {
        double dtmin = c->geo.sys[0].dt;
        for (const SysDesc &d : c->geo.sys) dtmin = std::min(dtmin, d.dt);
        for (size_t k = 0; k < c->geo.sys.size(); ++k) {
            const double ratio = c->geo.sys[k].dt / dtmin;
            const long long q = std::llround(ratio);
            if (q < 1 || q > 1024 || (q & (q - 1)) || std::fabs((double)q * dtmin - c->geo.sys[k].dt) > 1e-12 * c->geo.sys[k].dt)
                return fail(c, DEM_ERR_ARG, "multi-rate stepping needs every dt to be the smallest dt times a power of two (up to 1024)");
            stride[k] = (int32_t)q;
            mx = std::max(mx, (int32_t)q);
        }
    }
    for (size_t k = 0; k < c->geo.sys.size(); ++k) c->geo.sys[k].stride = stride[k];
    HIPCALL(c, hipMemcpyAsync(c->d_sys, c->geo.sys.data(), c->geo.sys.size() * sizeof(SysDesc), hipMemcpyHostToDevice,
                              c->stream));
    HIPCALL(c, hipStreamSynchronize(c->stream));
    c->multirate = enable != 0 && c->geo.sys.size() > 1;
    c->max_stride = c->multirate ? mx : 1;
    for (GraphSlot &gs : c->graphs) gs.chunk = 0;   // re-capture
    return upload_tiles(c);
}

int dem_set_step_options(dem_ctx *c, int use_graph, int32_t chunk) {
    if (!c) return DEM_ERR_ARG;
    if (chunk < 2 || chunk > 1024 || (chunk & 1)) return fail(c, DEM_ERR_ARG, "chunk must be even, 2..1024");
    c->use_graph = use_graph != 0;
    c->chunk = chunk;
    return DEM_OK;
}

int dem_set_launch(dem_ctx *c, int32_t lanes, int32_t max_blocks) {
    if (!c) return DEM_ERR_ARG;
    if (max_blocks < 0) return fail(c, DEM_ERR_ARG, "max_blocks must be >= 0");
    if (lanes == 0) lanes = default_lanes(c->geo.n, c->geo.block);
    if (lanes != 4 && lanes != 8 && lanes != 16) return fail(c, DEM_ERR_ARG, "lanes must be 0, 4, 8 or 16");
    if (lanes > c->geo.block) return fail(c, DEM_ERR_ARG, "lanes must not exceed the block size");
    c->grid_cap = max_blocks;
    c->lanes = lanes;
    for (GraphSlot &g : c->graphs) g.chunk = 0;  // re-capture with the new grid/lanes
    c->cpl_key.clear();                          // and the coupled interval's graph
    return upload_tiles(c);
}

int dem_step(dem_ctx *c, const dem_state *s, int64_t nsteps) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (nsteps < 0) return fail(c, DEM_ERR_ARG, "nsteps < 0");
    if (!c->masses) return fail(c, DEM_ERR_STATE, "dem_reset first");
    if (!c->forces_valid)
        return fail(c, DEM_ERR_STATE,
                    "dem_step needs the forces of the current state: call dem_forces(ctx, s, 0) or dem_declare_forces");
    if (nsteps == 0 || c->geo.n == 0) return DEM_OK;
    if (c->multirate && nsteps % c->max_stride)
        return fail(c, DEM_ERR_ARG, "multi-rate stepping needs nsteps to be a multiple of the largest stride");
    if (!c->list_current) {
        // binned but no list yet: build it (f and t were permuted with the particles)
        if ((rc = do_bin(c, s, true)) || (rc = do_neighbors(c, s))) return rc;
    }
    const int64_t base = c->step_counter;
    Flags h;
    HIPCALL(c, launch_ctrl(c->d_flags, 0, base + 1, c->stream));
    if (c->multirate) {
        HIPCALL(c, launch_ctrl(c->d_flags, 5, base, c->stream));
        HIPCALL(c, launch_ctrl(c->d_flags, 6, base + nsteps, c->stream));
    }
    {
        KArgs a = kargs(c, s);
        if ((rc = tic(c, 0))) return rc;
        HIPCALL(c, launch_pack(a, 0, 1, 0, 1, c->stream));
        if ((rc = toc(c))) return rc;
    }
    if ((rc = step_loop(c, s, nsteps, base, 1, h))) return rc;
    // the flags read after the last group are final: its last launch counted the steps
    if ((rc = collect_times(c))) return rc;
    c->step_counter += nsteps;
    c->binned = false;
    c->forces_valid = true;
    return flag_error(c, h);
}

int dem_set_timing(dem_ctx *c, int enable) {
    if (!c) return DEM_ERR_ARG;
    c->timing = enable != 0;
    for (int k = 0; k < kKinds; ++k) { c->t_ms[k] = 0.0; c->t_n[k] = 0; }
    c->ev_used = 0;
    return DEM_OK;
}

int dem_kernel_times(dem_ctx *c, double ms[4], int64_t launches[4]) {
    if (!c || !ms || !launches) return DEM_ERR_ARG;
    HIPCALL(c, hipStreamSynchronize(c->stream));
    int rc = collect_times(c);
    if (rc) return rc;
    for (int k = 0; k < kKinds; ++k) { ms[k] = c->t_ms[k]; launches[k] = c->t_n[k]; }
    return DEM_OK;
}

int dem_check(dem_ctx *c, int64_t info[4]) {
    if (!c) return DEM_ERR_ARG;
    Flags h;
    int rc = read_flags(c, h);
    if (rc) return rc;
    if (info) {
        info[0] = h.err;
        info[1] = h.max_row;
        info[2] = h.builds;
        info[3] = h.steps;
    }
    return flag_error(c, h);
}

int dem_stats(dem_ctx *c, int64_t out[5]) {
    if (!c || !out) return DEM_ERR_ARG;
    Flags h;
    int rc = read_flags(c, h);
    if (rc) return rc;
    out[0] = h.steps;
    out[1] = h.builds;
    out[2] = (int64_t)h.contacts;
    out[3] = (int64_t)h.wall_contacts;
    int64_t slots = 0;
    if (c->have_list && c->geo.n > 0) {
        std::vector<int32_t> cnt[2], cur(c->geo.sys.size());
        for (int b = 0; b < 2; ++b) {
            cnt[b].resize(c->geo.n);
            HIPCALL(c, hipMemcpy(cnt[b].data(), c->lists[b].cnt, c->geo.n * 4, hipMemcpyDeviceToHost));
        }
        HIPCALL(c, hipMemcpy(cur.data(), c->ws + c->lay.lcur, cur.size() * 4, hipMemcpyDeviceToHost));
        for (size_t sy = 0; sy < c->geo.sys.size(); ++sy)
            for (int64_t i = c->geo.sys[sy].p0; i < c->geo.sys[sy].pe; ++i) slots += cnt[cur[sy] & 1][i];
    }
    out[4] = slots;
    return DEM_OK;
}

// ------------------------------------------------------------ host exports

namespace {

struct HostList {
    std::vector<uint8_t> which, live;
    std::vector<int32_t> nbr, cnt, ids, id_now;
    std::vector<uint64_t> mask;
    std::vector<double> xi, x, r, xiw;
};

// Host copy of every system's current list (rows taken from the buffer each
// system currently uses).  `which` records that buffer per particle.
int fetch_list(dem_ctx *c, const dem_state *s, HostList &H, bool with_xi, bool with_pos) {
    const int64_t n = c->geo.n, K = c->geo.kmax;
    HIPCALL(c, hipStreamSynchronize(c->stream));
    std::vector<int32_t> cur(c->geo.sys.size());
    HIPCALL(c, hipMemcpy(cur.data(), c->ws + c->lay.lcur, cur.size() * 4, hipMemcpyDeviceToHost));
    H.which.assign(n, 0);
    H.live.assign(n, 0);
    for (size_t sy = 0; sy < c->geo.sys.size(); ++sy)
        for (int64_t i = c->geo.sys[sy].p0; i < c->geo.sys[sy].p1; ++i) {
            H.which[i] = (uint8_t)(cur[sy] & 1);
            H.live[i] = i < c->geo.sys[sy].pe ? 1 : 0;
        }
    H.nbr.resize(K * n);
    H.cnt.resize(n);
    H.ids.resize(n);
    H.mask.resize(n);
    if (with_xi) H.xi.resize(4 * K * n);
    for (int b = 0; b < 2; ++b) {
        const List &L = c->lists[b];
        std::vector<int32_t> nbr(K * n), cnt(n), ids(n);
        std::vector<uint64_t> mask(n);
        std::vector<double> xi;
        HIPCALL(c, hipMemcpy(nbr.data(), L.nbr, K * n * 4, hipMemcpyDeviceToHost));
        HIPCALL(c, hipMemcpy(cnt.data(), L.cnt, n * 4, hipMemcpyDeviceToHost));
        HIPCALL(c, hipMemcpy(ids.data(), L.ids, n * 4, hipMemcpyDeviceToHost));
        HIPCALL(c, hipMemcpy(mask.data(), L.mask, n * 8, hipMemcpyDeviceToHost));
        if (with_xi) {
            xi.resize(4 * K * n);
            HIPCALL(c, hipMemcpy(xi.data(), L.xi, 4 * K * n * 8, hipMemcpyDeviceToHost));
        }
        for (int64_t i = 0; i < n; ++i) {
            if (H.which[i] != b) continue;
            if (!H.live[i]) {   // a free slot: no row
                H.cnt[i] = 0;
                H.ids[i] = -1;
                H.mask[i] = 0;
                continue;
            }
            H.cnt[i] = cnt[i];
            H.ids[i] = ids[i];
            H.mask[i] = mask[i];
            for (int64_t q = 0; q < K; ++q) H.nbr[i * K + q] = nbr[q * n + i];   // device: slot major
            if (with_xi)
                for (int64_t q = 0; q < 4 * K; ++q) H.xi[4 * K * i + q] = xi[4 * K * i + q];
        }
    }
    if (with_xi) {
        H.xiw.resize(3 * n);
        HIPCALL(c, hipMemcpy(H.xiw.data(), c->ws + c->lay.xiw, 3 * n * 8, hipMemcpyDeviceToHost));
    }
    if (with_pos) {
        H.x.resize(3 * n);
        H.r.resize(n);
        HIPCALL(c, hipMemcpy(H.x.data(), s->x, 3 * n * 8, hipMemcpyDeviceToHost));
        HIPCALL(c, hipMemcpy(H.r.data(), s->r, n * 8, hipMemcpyDeviceToHost));
    }
    return DEM_OK;
}

int sys_index(const Geometry &g, int64_t i) {
    for (size_t s = 0; s < g.sys.size(); ++s)
        if (i < g.sys[s].p1) return (int)s;
    return (int)g.sys.size() - 1;
}

}  // namespace

int dem_export_neighbors(dem_ctx *c, const dem_state *s, int32_t *id_i, int32_t *id_j, int64_t cap, int64_t *count) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!count) return fail(c, DEM_ERR_ARG, "count is NULL");
    if (!c->list_current) return fail(c, DEM_ERR_STATE, "no neighbour list for the current order");
    HostList H;
    if ((rc = fetch_list(c, s, H, false, false))) return rc;
    const int64_t n = c->geo.n;
    std::vector<std::pair<int32_t, int32_t>> out;
    for (int64_t i = 0; i < n; ++i)
        for (int q = 0; q < H.cnt[i]; ++q) out.push_back({H.ids[i], H.ids[H.nbr[i * c->geo.kmax + q]]});
    std::sort(out.begin(), out.end());
    *count = (int64_t)out.size();
    for (int64_t k = 0; k < *count && k < cap; ++k) {
        if (id_i) id_i[k] = out[k].first;
        if (id_j) id_j[k] = out[k].second;
    }
    Flags h;
    if ((rc = read_flags(c, h))) return rc;
    return flag_error(c, h);
}

int dem_export_contacts(dem_ctx *c, const dem_state *s, int32_t *id_i, int32_t *id_j, double *xi, int64_t cap,
                        int64_t *count) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!count) return fail(c, DEM_ERR_ARG, "count is NULL");
    if (!c->list_current) return fail(c, DEM_ERR_STATE, "no neighbour list for the current order");
    HostList H;
    if ((rc = fetch_list(c, s, H, true, true))) return rc;
    const int64_t n = c->geo.n, K = c->geo.kmax;
    struct Rec { int32_t a, b; double x, y, z; };
    std::vector<Rec> out;
    for (int64_t i = 0; i < n; ++i) {
        const SysDesc &sd = c->geo.sys[sys_index(c->geo, i)];
        for (int q = 0; q < H.cnt[i]; ++q) {
            const int64_t j = H.nbr[i * K + q];
            double dx = min_image(H.x[i] - H.x[j], sd.L[0], sd.hL[0], sd.periodic[0]);
            double dy = min_image(H.x[n + i] - H.x[n + j], sd.L[1], sd.hL[1], sd.periodic[1]);
            double dz = min_image(H.x[2 * n + i] - H.x[2 * n + j], sd.L[2], sd.hL[2], sd.periodic[2]);
            double d2 = dx * dx + dy * dy + dz * dz;
            double rs = H.r[i] + H.r[j];
            if (!(d2 < rs * rs)) continue;
            const int64_t rec = 4 * (i * K + q);
            Rec r{H.ids[i], H.ids[j], 0.0, 0.0, 0.0};
            if ((H.mask[i] >> q) & 1ull) { r.x = H.xi[rec]; r.y = H.xi[rec + 1]; r.z = H.xi[rec + 2]; }
            out.push_back(r);
        }
    }
    std::sort(out.begin(), out.end(), [](const Rec &p, const Rec &q) { return p.a != q.a ? p.a < q.a : p.b < q.b; });
    *count = (int64_t)out.size();
    for (int64_t k = 0; k < *count && k < cap; ++k) {
        if (id_i) id_i[k] = out[k].a;
        if (id_j) id_j[k] = out[k].b;
        if (xi) { xi[3 * k] = out[k].x; xi[3 * k + 1] = out[k].y; xi[3 * k + 2] = out[k].z; }
    }
    Flags h;
    if ((rc = read_flags(c, h))) return rc;
    return flag_error(c, h);
}

int dem_export_wall(dem_ctx *c, const dem_state *s, int32_t *id, double *xi, int64_t cap, int64_t *count) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!count) return fail(c, DEM_ERR_ARG, "count is NULL");
    if (!c->list_current) return fail(c, DEM_ERR_STATE, "no neighbour list for the current order");
    HostList H;
    if ((rc = fetch_list(c, s, H, true, true))) return rc;
    const int64_t n = c->geo.n;
    struct Rec { int32_t a; double x, y, z; };
    std::vector<Rec> out;
    for (int64_t i = 0; i < n; ++i) {
        const SysDesc &sd = c->geo.sys[sys_index(c->geo, i)];
        if (!H.live[i] || !sd.wall || !(H.x[2 * n + i] < H.r[i])) continue;
        Rec r{H.ids[i], 0.0, 0.0, 0.0};
        if (H.mask[i] & kWallBit) { r.x = H.xiw[i]; r.y = H.xiw[n + i]; r.z = H.xiw[2 * n + i]; }
        out.push_back(r);
    }
    std::sort(out.begin(), out.end(), [](const Rec &p, const Rec &q) { return p.a < q.a; });
    *count = (int64_t)out.size();
    for (int64_t k = 0; k < *count && k < cap; ++k) {
        if (id) id[k] = out[k].a;
        if (xi) { xi[3 * k] = out[k].x; xi[3 * k + 1] = out[k].y; xi[3 * k + 2] = out[k].z; }
    }
    return DEM_OK;
}

int dem_import_history(dem_ctx *c, const dem_state *s, int64_t npairs, const int32_t *id_i, const int32_t *id_j,
                       const double *xi, int64_t nwall, const int32_t *wall_id, const double *wall_xi) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (npairs < 0 || nwall < 0 || (npairs && (!id_i || !id_j || !xi)) || (nwall && (!wall_id || !wall_xi)))
        return fail(c, DEM_ERR_ARG, "bad history arrays");
    if (!c->list_current) return fail(c, DEM_ERR_STATE, "dem_import_history needs a neighbour list");
    HostList H;
    if ((rc = fetch_list(c, s, H, true, false))) return rc;
    const int64_t n = c->geo.n, K = c->geo.kmax;
    std::unordered_map<uint64_t, int64_t> pairs;
    pairs.reserve((size_t)npairs * 2);
    for (int64_t k = 0; k < npairs; ++k)
        pairs[((uint64_t)(uint32_t)id_i[k] << 32) | (uint32_t)id_j[k]] = k;
    std::unordered_map<int32_t, int64_t> walls;
    for (int64_t k = 0; k < nwall; ++k) walls[wall_id[k]] = k;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t m = 0;
        for (int q = 0; q < H.cnt[i]; ++q) {
            const int32_t a = H.ids[i], b = H.ids[H.nbr[i * K + q]];
            auto it = pairs.find(((uint64_t)(uint32_t)a << 32) | (uint32_t)b);
            double v[3] = {0.0, 0.0, 0.0};
            if (it != pairs.end()) for (int d = 0; d < 3; ++d) v[d] = xi[3 * it->second + d];
            for (int d = 0; d < 3; ++d) H.xi[4 * (i * K + q) + d] = v[d];
            H.xi[4 * (i * K + q) + 3] = 0.0;
            if (v[0] != 0.0 || v[1] != 0.0 || v[2] != 0.0) m |= 1ull << q;
        }
        auto w = H.live[i] ? walls.find(H.ids[i]) : walls.end();
        double v[3] = {0.0, 0.0, 0.0};
        if (w != walls.end()) for (int d = 0; d < 3; ++d) v[d] = wall_xi[3 * w->second + d];
        for (int d = 0; d < 3; ++d) H.xiw[d * n + i] = v[d];
        if (v[0] != 0.0 || v[1] != 0.0 || v[2] != 0.0) m |= kWallBit;
        H.mask[i] = m;
    }
    for (int b = 0; b < 2; ++b) {
        // rows of the particles whose system uses buffer b
        const List &L = c->lists[b];
        std::vector<double> xi(4 * K * n);
        std::vector<uint64_t> mask(n);
        HIPCALL(c, hipMemcpy(xi.data(), L.xi, 4 * K * n * 8, hipMemcpyDeviceToHost));
        HIPCALL(c, hipMemcpy(mask.data(), L.mask, n * 8, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            if (H.which[i] != b) continue;
            mask[i] = H.mask[i];
            for (int64_t q = 0; q < 4 * K; ++q) xi[4 * K * i + q] = H.xi[4 * K * i + q];
        }
        HIPCALL(c, hipMemcpy(L.xi, xi.data(), 4 * K * n * 8, hipMemcpyHostToDevice));
        HIPCALL(c, hipMemcpy(L.mask, mask.data(), n * 8, hipMemcpyHostToDevice));
    }
    HIPCALL(c, hipMemcpy(c->ws + c->lay.xiw, H.xiw.data(), 3 * n * 8, hipMemcpyHostToDevice));
    return DEM_OK;
}

int dem_export_surface_history(dem_ctx *c, const dem_state *s, int32_t *id, int32_t *surf, double *xi, int64_t cap,
                               int64_t *count) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!count) return fail(c, DEM_ERR_ARG, "count is NULL");
    *count = 0;
    const int64_t n = c->geo.n;
    const int S = c->geo.nsurf_slots;
    if (S == 0 || n == 0) return DEM_OK;
    HIPCALL(c, hipStreamSynchronize(c->stream));
    std::vector<uint32_t> mask((size_t)n);
    std::vector<D4> h((size_t)S * n);
    std::vector<int32_t> ids((size_t)n);
    HIPCALL(c, hipMemcpy(mask.data(), c->ws + c->lay.smask, (size_t)n * 4, hipMemcpyDeviceToHost));
    HIPCALL(c, hipMemcpy(h.data(), c->ws + c->lay.sxi, (size_t)S * n * sizeof(D4), hipMemcpyDeviceToHost));
    HIPCALL(c, hipMemcpy(ids.data(), s->id, (size_t)n * 4, hipMemcpyDeviceToHost));
    struct Rec { int32_t a, k; double x, y, z; };
    std::vector<Rec> out;
    for (int64_t i = 0; i < n; ++i) {
        const SysDesc &sd = c->geo.sys[sys_index(c->geo, i)];
        if (i >= sd.pe) continue;
        for (int k = 0; k < sd.nsurf; ++k)
            if ((mask[i] >> k) & 1u) {
                const D4 &v = h[(size_t)k * n + i];
                out.push_back(Rec{ids[i], k, v.x, v.y, v.z});
            }
    }
    std::sort(out.begin(), out.end(), [](const Rec &p, const Rec &q) { return p.a != q.a ? p.a < q.a : p.k < q.k; });
    *count = (int64_t)out.size();
    for (int64_t k = 0; k < *count && k < cap; ++k) {
        if (id) id[k] = out[k].a;
        if (surf) surf[k] = out[k].k;
        if (xi) { xi[3 * k] = out[k].x; xi[3 * k + 1] = out[k].y; xi[3 * k + 2] = out[k].z; }
    }
    return DEM_OK;
}

int dem_import_surface_history(dem_ctx *c, const dem_state *s, int64_t count, const int32_t *id, const int32_t *surf,
                               const double *xi) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (count < 0 || (count && (!id || !surf || !xi))) return fail(c, DEM_ERR_ARG, "bad surface history arrays");
    const int64_t n = c->geo.n;
    const int S = c->geo.nsurf_slots;
    if (S == 0 || n == 0) return count ? fail(c, DEM_ERR_ARG, "no surfaces reserved") : DEM_OK;
    HIPCALL(c, hipStreamSynchronize(c->stream));
    std::vector<int32_t> ids((size_t)n);
    HIPCALL(c, hipMemcpy(ids.data(), s->id, (size_t)n * 4, hipMemcpyDeviceToHost));
    std::unordered_map<int32_t, int64_t> where;
    for (int64_t i = 0; i < n; ++i)
        if (i < c->geo.sys[sys_index(c->geo, i)].pe) where[ids[i]] = i;
    std::vector<uint32_t> mask((size_t)n, 0u);
    std::vector<D4> h((size_t)S * n, D4{0.0, 0.0, 0.0, 0.0});
    for (int64_t r = 0; r < count; ++r) {
        auto it = where.find(id[r]);
        if (it == where.end()) return fail(c, DEM_ERR_ARG, "surface history of an id that is not live");
        const int64_t i = it->second;
        const int k = surf[r];
        if (k < 0 || k >= c->geo.sys[sys_index(c->geo, i)].nsurf)
            return fail(c, DEM_ERR_ARG, "surface index out of range for the sphere's system");
        const double x = xi[3 * r], y = xi[3 * r + 1], z = xi[3 * r + 2];
        h[(size_t)k * n + i] = D4{x, y, z, 0.0};
        if (x != 0.0 || y != 0.0 || z != 0.0) mask[i] |= 1u << k;
    }
    HIPCALL(c, hipMemcpy(c->ws + c->lay.sxi, h.data(), (size_t)S * n * sizeof(D4), hipMemcpyHostToDevice));
    HIPCALL(c, hipMemcpy(c->ws + c->lay.smask, mask.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    return DEM_OK;
}

const char *dem_last_error(const dem_ctx *c) { return c ? c->err.c_str() : g_init_error.c_str(); }

int dem_destroy(dem_ctx *c) {
    if (!c) return DEM_ERR_ARG;
    if (c->static_dev >= 0) {
        // later contexts may reuse the array once this one's work is done
        (void)hipStreamSynchronize(c->stream);
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
    }
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (GraphSlot &g : c->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (c->cpl_exec) (void)hipGraphExecDestroy(c->cpl_exec);
    if (c->h_flags) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipHostFree(c->h_flags);
    }
    delete c;
    return DEM_OK;
}

}  // extern "C"
