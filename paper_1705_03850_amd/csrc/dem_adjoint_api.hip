// dem_adjoint_api.hip -- host side of the reverse-mode rollout and of the
// material-parameter calls declared in include/dem.h.
//
// Forward: the fused step of the plain path advances the rollout in windows;
// a list rebuild is only allowed between windows, so inside each window the
// neighbour list (the contact topology) is fixed.  At the start of every
// window the packed state and the slot history are checkpointed; after a
// rebuild also the new list and the permutation to the previous order.
// Backward: windows in reverse order; each is recomputed from its checkpoint
// (all its evaluations' inputs kept), then reversed evaluation by evaluation,
// and the adjoint is carried across the rebuild to the previous window.
// Kept mode: the forward runs the evaluation kernel of the reverse pass in
// its gated form and stores the inputs of every evaluation, so the backward
// recomputes nothing (memory grows with the step count instead of the window).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "dem_adjoint.h"
#include "dem_ctx.h"

using namespace dem;
using namespace dem::host;

namespace {

struct Topo {
    size_t nbr, cnt, ids, frame, im;
};
struct Ckpt {
    size_t pos, vel, spin, hist, hw;
    int topo = 0;
    int rebuilt = 0;
    int64_t q0 = 0;
    int32_t len = 0;
};
struct StepBuf {
    size_t pos, vel, spin, hist, hw;
};

}  // namespace

struct dem_adjoint {
    dem_ctx *ctx = nullptr;
    int64_t nsteps = 0;
    int32_t window = 0, max_windows = 0;
    char *ws = nullptr;
    size_t bytes = 0;
    std::vector<Ckpt> ck;         // slot 0: state before the rollout; 1..: window starts
    std::vector<Topo> topo;
    std::vector<StepBuf> traj;    // inputs of a window's evaluations 2..len
    size_t rec[2] = {0, 0}, mu[2] = {0, 0}, muw[2] = {0, 0}, gp = 0, acc = 0, part = 0, rowmax = 0;
    int32_t kslots = 0;           // history slots per particle in the adjoint's own buffers
    int32_t lanes = 4;
    int32_t keep = 0;             // every evaluation's inputs stored by the forward
    int nck = 0, ntopo = 0;
    int64_t step_end = -1;        // the context's step counter after the last forward
    int64_t rebuilds = 0;
};

namespace {

struct AdjLayout {
    std::vector<Ckpt> ck;
    std::vector<Topo> topo;
    std::vector<StepBuf> traj;
    size_t rec[2], mu[2], muw[2], gp, acc, part, rowmax, total;
};

// K: history slots per particle (kslots); rows of the saved lists hold K
// neighbour indices as well (the slot-major prefix of the live list).
AdjLayout adj_layout(int64_t n, int64_t K, int64_t nsteps, int32_t window, int32_t max_windows, int nt, int keep) {
    AdjLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    const size_t N = (size_t)n;
    const size_t rec = N * sizeof(D4), slots = N * (size_t)K * sizeof(D4);
    L.ck.resize((size_t)max_windows + 1);
    for (size_t k = 0; k < (keep ? 1 : L.ck.size()); ++k) {
        Ckpt &c = L.ck[k];
        c.pos = take(rec); c.vel = take(rec); c.spin = take(rec);
        c.hist = take(slots); c.hw = take(rec);
    }
    L.topo.resize((size_t)max_windows + 1);
    for (Topo &t : L.topo) {
        t.nbr = take(N * (size_t)K * 4); t.cnt = take(N * 4); t.ids = take(N * 4); t.frame = take(N * 4);
        t.im = take(N * sizeof(D2));
    }
    // kept: slot q - 1 holds the inputs of evaluation q, slot nsteps the final history
    L.traj.resize(keep ? (size_t)nsteps + 1 : window > 1 ? (size_t)window - 1 : 0);
    for (StepBuf &b : L.traj) {
        b.pos = take(rec); b.vel = take(rec); b.spin = take(rec);
        b.hist = take(slots); b.hw = take(rec);
    }
    for (int k = 0; k < 2; ++k) {
        L.rec[k] = take(5 * rec);
        L.mu[k] = take(slots);
        L.muw[k] = take(rec);
    }
    L.gp = take(N * 5 * (size_t)nt * 8);
    L.acc = take(5 * (size_t)nt * (size_t)nt * 8);
    L.part = take(adj_reduce_scratch_bytes(nt));
    L.rowmax = take(sizeof(int32_t));
    L.total = o;
    return L;
}

int32_t default_windows(int64_t nsteps, int32_t window) {
    const int64_t w = (nsteps + window - 1) / window;
    return (int32_t)std::min<int64_t>(2 * w + 1, 1 << 20);
}

int adj_args(dem_ctx *c, int64_t nsteps, int32_t window, int32_t &max_windows, int32_t &kslots) {
    if (!c) return DEM_ERR_ARG;
    if (kslots == 0) kslots = c->geo.kmax;
    if (kslots < 1 || kslots > c->geo.kmax) return fail(c, DEM_ERR_ARG, "kslots must be in 1..k_max (0: k_max)");
    if (c->geo.sys.size() != 1) return fail(c, DEM_ERR_ARG, "the adjoint rollout takes a context of one system");
    if (c->geo.sys[0].p1 != c->geo.sys[0].pe)
        return fail(c, DEM_ERR_ARG, "the adjoint rollout takes a system without free slots");
    if (nsteps < 1) return fail(c, DEM_ERR_ARG, "nsteps must be >= 1");
    if (window < 1 || window > 4096) return fail(c, DEM_ERR_ARG, "window must be in 1..4096");
    if (max_windows == 0) max_windows = default_windows(nsteps, window);
    if (max_windows < (nsteps + window - 1) / window)
        return fail(c, DEM_ERR_ARG, "max_windows must be at least ceil(nsteps / window)");
    return DEM_OK;
}

template <class T>
T *at(dem_adjoint *A, size_t off) {
    return (T *)(A->ws + off);
}

AArgs base_args(dem_adjoint *A) {
    dem_ctx *c = A->ctx;
    AArgs a;
    memset(&a, 0, sizeof a);
    a.n = c->geo.n;
    a.kmax = c->geo.kmax;
    a.kslots = A->kslots;
    a.ntypes = c->geo.sys[0].ntypes;
    a.sys = c->d_sys;
    a.coef = c->d_coef + c->geo.sys[0].coef0;
    a.seed_scale = 1.0;
    a.lanes = A->lanes;
    return a;
}

int fill_zero(dem_adjoint *A, size_t off, size_t doubles) {
    HIPCALL(A->ctx, launch_fill_f64(at<double>(A, off), (int64_t)doubles, 0.0, A->ctx->stream));
    return DEM_OK;
}

// The live list's longest row must fit the adjoint's kslots history slots:
// DEM_ERR_CAPACITY otherwise (checked before anything is written with the list).
int check_rows(dem_adjoint *A, const List &live) {
    dem_ctx *c = A->ctx;
    if (A->kslots >= c->geo.kmax) return DEM_OK;   // a build never leaves a row longer than k_max
    int32_t *d = at<int32_t>(A, A->rowmax);
    HIPCALL(c, launch_fill_i32(d, 1, 0, c->stream));
    HIPCALL(c, launch_adj_row_max(live.cnt, c->geo.n, d, c->stream));
    int32_t h = 0;
    HIPCALL(c, hipStreamSynchronize(c->stream));
    HIPCALL(c, hipMemcpy(&h, d, sizeof h, hipMemcpyDeviceToHost));
    if (h > A->kslots) {
        char buf[160];
        snprintf(buf, sizeof buf, "a neighbour row of %d entries exceeds the adjoint's kslots = %d", h, A->kslots);
        return fail(c, DEM_ERR_CAPACITY, buf);
    }
    return DEM_OK;
}

// Topology slot t from the live list (and the permutation written by the last bin).
int save_topology(dem_adjoint *A, const List &live, int t, bool with_frame) {
    dem_ctx *c = A->ctx;
    const size_t n = (size_t)c->geo.n, K = (size_t)A->kslots;
    const Topo &T = A->topo[t];
    hipStream_t st = c->stream;
    HIPCALL(c, hipMemcpyAsync(A->ws + T.nbr, live.nbr, n * K * 4, hipMemcpyDeviceToDevice, st));
    HIPCALL(c, hipMemcpyAsync(A->ws + T.cnt, live.cnt, n * 4, hipMemcpyDeviceToDevice, st));
    HIPCALL(c, hipMemcpyAsync(A->ws + T.ids, live.ids, n * 4, hipMemcpyDeviceToDevice, st));
    if (with_frame)
        HIPCALL(c, hipMemcpyAsync(A->ws + T.frame, c->ws + c->lay.frame, n * 4, hipMemcpyDeviceToDevice, st));
    HIPCALL(c, hipMemcpyAsync(A->ws + T.im, c->ws + c->lay.im, n * sizeof(D2), hipMemcpyDeviceToDevice, st));
    return DEM_OK;
}

// Packed buffer `buf` of the context and the live history -> the state record
// at the given offsets.
int save_state(dem_adjoint *A, const List &live, int buf, size_t pos, size_t vel, size_t spin, size_t hist,
               size_t hw) {
    dem_ctx *c = A->ctx;
    const size_t n = (size_t)c->geo.n;
    hipStream_t st = c->stream;
    HIPCALL(c, hipMemcpyAsync(A->ws + pos, c->ws + c->lay.pos[buf], n * sizeof(D4), hipMemcpyDeviceToDevice, st));
    HIPCALL(c, hipMemcpyAsync(A->ws + vel, c->ws + c->lay.vel[buf], n * sizeof(D4), hipMemcpyDeviceToDevice, st));
    HIPCALL(c, hipMemcpyAsync(A->ws + spin, c->ws + c->lay.spin[buf], n * sizeof(D4), hipMemcpyDeviceToDevice, st));
    AArgs a = base_args(A);
    a.cnt = live.cnt;
    HIPCALL(c, launch_adj_expand(a, live.xi, live.mask, (const double *)(c->ws + c->lay.xiw), at<D4>(A, hist),
                                 at<D4>(A, hw), st));
    return DEM_OK;
}

// Checkpoint slot k.  Stored: packed buffer `buf` of the context and the live
// history; kept mode (k >= 1): the record of evaluation q0's inputs, written
// here when `buf` >= 0 and by the previous window's last evaluation otherwise.
int save_checkpoint(dem_adjoint *A, const List &live, int k, int buf, int topo, int rebuilt, int64_t q0) {
    Ckpt &C = A->ck[k];
    if (A->keep && k >= 1) {
        const StepBuf &B = A->traj[(size_t)q0 - 1];
        C.pos = B.pos; C.vel = B.vel; C.spin = B.spin; C.hist = B.hist; C.hw = B.hw;
    }
    if (buf >= 0) {
        int rc = save_state(A, live, buf, C.pos, C.vel, C.spin, C.hist, C.hw);
        if (rc) return rc;
    }
    C.topo = topo;
    C.rebuilt = rebuilt;
    C.q0 = q0;
    C.len = 0;
    return DEM_OK;
}

// The state Y_q in packed buffer b needs a new list: rebuild on the caller's
// arrays and repack into buffer 0 (no kick: the evaluation of Y_q comes next).
int rebuild(dem_adjoint *A, const dem_state *s, int b) {
    dem_ctx *c = A->ctx;
    KArgs K = kargs(c, s);
    HIPCALL(c, launch_unpack(K, b, 0, c->stream));
    c->binned = false;
    int rc;
    if ((rc = do_bin(c, s, true)) || (rc = do_neighbors(c, s))) return rc;
    KArgs K2 = kargs(c, s);
    HIPCALL(c, launch_pack(K2, 0, 0, 0, 0, c->stream));
    ++A->rebuilds;
    return DEM_OK;
}

// Kept mode: the live list takes the history of state record B (written in
// the list's order), and, with `rebuild`, the list is rebuilt on B's state
// as above.
int restore_from(dem_adjoint *A, const dem_state *s, const List &live, const StepBuf &B, bool rebuild_list) {
    dem_ctx *c = A->ctx;
    AArgs a = base_args(A);
    a.cnt = live.cnt;
    a.pos = at<D4>(A, B.pos); a.vel = at<D4>(A, B.vel); a.spin = at<D4>(A, B.spin);
    HIPCALL(c, launch_adj_compress(a, at<D4>(A, B.hist), at<D4>(A, B.hw), live.xi, live.mask,
                                   (double *)(c->ws + c->lay.xiw), c->stream));
    if (!rebuild_list) return DEM_OK;
    HIPCALL(c, launch_adj_unpack(a, s->x, s->v, s->w, c->stream));
    c->binned = false;
    int rc;
    if ((rc = do_bin(c, s, true)) || (rc = do_neighbors(c, s))) return rc;
    KArgs K2 = kargs(c, s);
    HIPCALL(c, launch_pack(K2, 0, 0, 0, 0, c->stream));
    ++A->rebuilds;
    return DEM_OK;
}

// Coefficient adjoints G[ti][tj][kn0, kt0, gn0, gt0, mu] -> dL/dE, dL/de, dL/dmu
// per type, through the folded Eq. (6): k_n0 = 4/3 E*, k_t0 = 8 G*,
// g_n0 = -beta sqrt(20/3 E*), g_t0 = -beta sqrt(80/3 G*), E* and G* harmonic,
// e and mu arithmetic means of the two types, beta = ln e / sqrt(ln^2 e + pi^2).
void chain_rule(const dem_ctx *c, const double *G, double *grad) {
    const SysDesc &sd = c->geo.sys[0];
    const int nt = sd.ntypes;
    const dem_material *m = &c->geo.mat[sd.type0];
    for (int k = 0; k < 3 * nt; ++k) grad[k] = 0.0;
    for (int ti = 0; ti < nt; ++ti)
        for (int tj = 0; tj < nt; ++tj) {
            const double *g = G + (ti * nt + tj) * 5;
            const dem_material &A = m[ti], &B = m[tj];
            const double aE = (1.0 - A.nu * A.nu) / A.E, bE = (1.0 - B.nu * B.nu) / B.E;
            const double aG = 2.0 * (2.0 - A.nu) * (1.0 + A.nu) / A.E, bG = 2.0 * (2.0 - B.nu) * (1.0 + B.nu) / B.E;
            const double Es = 1.0 / (aE + bE), Gs = 1.0 / (aG + bG);
            const double e = (A.e + B.e) / 2.0, le = std::log(e), D = le * le + M_PI * M_PI;
            const double beta = le / std::sqrt(D);
            const double dbeta = M_PI * M_PI / (e * D * std::sqrt(D));
            const double sEn = std::sqrt(20.0 / 3.0 * Es), sGt = std::sqrt(80.0 / 3.0 * Gs);
            const double gEs = g[0] * (4.0 / 3.0) + g[2] * (-beta * (10.0 / 3.0) / sEn);
            const double gGs = g[1] * 8.0 + g[3] * (-beta * (40.0 / 3.0) / sGt);
            const double gbeta = g[2] * -sEn + g[3] * -sGt;
            grad[ti] += gEs * Es * Es * aE / A.E + gGs * Gs * Gs * aG / A.E;
            grad[tj] += gEs * Es * Es * bE / B.E + gGs * Gs * Gs * bG / B.E;
            grad[nt + ti] += 0.5 * gbeta * dbeta;
            grad[nt + tj] += 0.5 * gbeta * dbeta;
            grad[2 * nt + ti] += 0.5 * g[4];
            grad[2 * nt + tj] += 0.5 * g[4];
        }
}

int finish_grad(dem_adjoint *A, double *grad) {
    dem_ctx *c = A->ctx;
    const int nt = c->geo.sys[0].ntypes;
    std::vector<double> G((size_t)5 * nt * nt);
    HIPCALL(c, hipStreamSynchronize(c->stream));
    HIPCALL(c, hipMemcpy(G.data(), A->ws + A->acc, G.size() * 8, hipMemcpyDeviceToHost));
    if (grad) chain_rule(c, G.data(), grad);
    return DEM_OK;
}

}  // namespace

extern "C" {

int dem_set_materials(dem_ctx *c, int32_t sys, const dem_material *mat, int32_t ntypes) {
    if (!c || !mat) return DEM_ERR_ARG;
    if (sys < 0 || sys >= (int32_t)c->geo.sys.size()) return fail(c, DEM_ERR_ARG, "system index out of range");
    const SysDesc &sd = c->geo.sys[sys];
    if (ntypes != sd.ntypes) return fail(c, DEM_ERR_ARG, "ntypes differs from the system's");
    for (int t = 0; t < ntypes; ++t) {
        if (!material_ok(mat[t])) return fail(c, DEM_ERR_ARG, "need E > 0, -1 < nu < 0.5, rho > 0, 0 < e <= 1, mu >= 0");
        if (mat[t].rho != c->geo.mat[sd.type0 + t].rho) return fail(c, DEM_ERR_ARG, "rho is fixed after init");
    }
    for (int t = 0; t < ntypes; ++t) c->geo.mat[sd.type0 + t] = mat[t];
    for (int ti = 0; ti < ntypes; ++ti)
        for (int tj = 0; tj < ntypes; ++tj) c->geo.coef[sd.coef0 + ti * ntypes + tj] = pair_coef(mat[ti], mat[tj]);
    HIPCALL(c, hipMemcpyAsync(c->d_coef + sd.coef0, c->geo.coef.data() + sd.coef0,
                              (size_t)ntypes * ntypes * sizeof(PairCoef), hipMemcpyHostToDevice, c->stream));
    HIPCALL(c, hipStreamSynchronize(c->stream));
    c->forces_valid = false;   // the stored forces belong to the old materials
    return DEM_OK;
}

int dem_adjoint_workspace_size(dem_ctx *c, int64_t nsteps, int32_t window, int32_t max_windows, int32_t keep,
                               int32_t kslots, size_t *bytes) {
    if (!bytes) return DEM_ERR_ARG;
    int rc = adj_args(c, nsteps, window, max_windows, kslots);
    if (rc) return rc;
    *bytes = adj_layout(c->geo.n, kslots, nsteps, window, max_windows, c->geo.sys[0].ntypes, keep != 0).total;
    return DEM_OK;
}

int dem_adjoint_init(dem_ctx *c, int64_t nsteps, int32_t window, int32_t max_windows, int32_t keep, int32_t kslots,
                     void *workspace, size_t bytes, dem_adjoint **out) {
    if (!out) return DEM_ERR_ARG;
    *out = nullptr;
    int rc = adj_args(c, nsteps, window, max_windows, kslots);
    if (rc) return rc;
    AdjLayout L = adj_layout(c->geo.n, kslots, nsteps, window, max_windows, c->geo.sys[0].ntypes, keep != 0);
    if (!workspace || bytes < L.total) return fail(c, DEM_ERR_ARG, "adjoint workspace too small");
    if ((uintptr_t)workspace % kAlign) return fail(c, DEM_ERR_ARG, "adjoint workspace must be 256-byte aligned");
    dem_adjoint *A = new dem_adjoint();
    A->ctx = c;
    A->nsteps = nsteps;
    A->window = window;
    A->max_windows = max_windows;
    A->keep = keep != 0;
    A->kslots = kslots;
    A->ws = (char *)workspace;
    A->bytes = bytes;
    A->ck = L.ck;
    A->topo = L.topo;
    A->traj = L.traj;
    for (int k = 0; k < 2; ++k) { A->rec[k] = L.rec[k]; A->mu[k] = L.mu[k]; A->muw[k] = L.muw[k]; }
    A->gp = L.gp;
    A->acc = L.acc;
    A->part = L.part;
    A->rowmax = L.rowmax;
    *out = A;
    return DEM_OK;
}

int dem_rollout_forward(dem_adjoint *A, const dem_state *s) {
    if (!A) return DEM_ERR_ARG;
    dem_ctx *c = A->ctx;
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!c->masses) return fail(c, DEM_ERR_STATE, "dem_reset first");
    if (c->fext_on) return fail(c, DEM_ERR_STATE, "the reverse mode does not take external forces");
    if (c->geo.sys[0].pe != c->geo.sys[0].p1)
        return fail(c, DEM_ERR_STATE, "the reverse mode takes a system without free slots");
    A->nck = 0;
    A->ntopo = 0;
    A->rebuilds = 0;
    A->step_end = -1;
    if (c->geo.n == 0) return DEM_ERR_STATE;
    if (!c->list_current)
        if ((rc = do_bin(c, s, true)) || (rc = do_neighbors(c, s))) return rc;
    const int64_t S = A->nsteps, base = c->step_counter;
    const int cnt = c->count ? 1 : 0;
    List live;
    if ((rc = live_list(c, 0, live)) || (rc = check_rows(A, live))) return rc;
    KArgs K = kargs(c, s);
    // slot 0: the state before the rollout and its first force evaluation
    HIPCALL(c, launch_pack(K, 0, 0, 0, 0, c->stream));
    if ((rc = save_topology(A, live, 0, false))) return rc;
    if ((rc = save_checkpoint(A, live, 0, 0, 0, 0, 0))) return rc;
    HIPCALL(c, launch_step(K, 0, 0, 0, 0, 0, c->stream));
    HIPCALL(c, launch_ctrl(c->d_flags, 0, base + 1, c->stream));
    HIPCALL(c, launch_pack(K, 0, 1, 0, 1, c->stream));       // kick + drift into Y_1
    A->nck = 1;
    A->ntopo = 1;
    Flags h;
    if ((rc = read_flags(c, h)) || (rc = flag_error(c, h))) return rc;
    int64_t q = 1;
    int buf = 0, rebuilt = 0;
    if (h.abort_at != INT64_MAX) {
        if ((rc = rebuild(A, s, 0))) return rc;
        rebuilt = 1;
    }
    while (q <= S) {
        if (A->nck > A->max_windows)
            return fail(c, DEM_ERR_CAPACITY, "the rollout needs more windows than max_windows (list rebuilds split windows)");
        if (rebuilt) {
            if ((rc = live_list(c, 0, live)) || (rc = check_rows(A, live))) return rc;
            if ((rc = save_topology(A, live, A->ntopo, true))) return rc;
            ++A->ntopo;
        }
        const bool fresh = !A->keep || q == 1 || rebuilt;   // kept: else written by the last evaluation
        if ((rc = save_checkpoint(A, live, A->nck, fresh ? buf : -1, A->ntopo - 1, rebuilt, q))) return rc;
        const int len = (int)std::min<int64_t>(A->window, S - q + 1);
        HIPCALL(c, launch_ctrl(c->d_flags, 0, base + q, c->stream));
        if (A->keep) {
            const Topo &T = A->topo[A->ntopo - 1];
            AArgs a = base_args(A);
            a.nbr = at<int32_t>(A, T.nbr);
            a.cnt = at<int32_t>(A, T.cnt);
            a.im = K.im;
            a.flags = c->d_flags;
            a.disp = K.disp;
            a.x = s->x; a.v = s->v; a.w = s->w; a.f = s->f; a.t = s->t;
            for (int k = 0; k < len; ++k) {
                const StepBuf &I = A->traj[(size_t)(q + k) - 1], &O = A->traj[(size_t)(q + k)];
                a.pos = at<D4>(A, I.pos); a.vel = at<D4>(A, I.vel); a.spin = at<D4>(A, I.spin);
                a.hin = at<D4>(A, I.hist); a.hwin = at<D4>(A, I.hw);
                a.pos_o = at<D4>(A, O.pos); a.vel_o = at<D4>(A, O.vel); a.spin_o = at<D4>(A, O.spin);
                a.hout = at<D4>(A, O.hist); a.hwout = at<D4>(A, O.hw);
                a.k = k;
                HIPCALL(c, launch_adj_forward(a, q + k == S ? 2 : 1, c->stream));
            }
        } else {
            for (int k = 0; k < len; ++k)
                HIPCALL(c, launch_step(K, buf ^ (k & 1), q + k == S ? 2 : 1, k, 1, cnt, c->stream));
        }
        if ((rc = read_flags(c, h)) || (rc = flag_error(c, h))) return rc;
        Ckpt &C = A->ck[A->nck];
        if (h.abort_at != INT64_MAX) {
            const int64_t qa = h.abort_at - base;   // the first evaluation that needs the new list
            if (qa <= q || qa > q + len) return fail(c, DEM_ERR_STATE, "rebuild request outside the window");
            C.len = (int32_t)(qa - q);
            if (A->keep) rc = restore_from(A, s, live, A->traj[(size_t)qa - 1], true);
            else rc = rebuild(A, s, buf ^ (int)((qa - q) & 1));
            if (rc) return rc;
            buf = 0;
            rebuilt = 1;
            q = qa;
        } else {
            C.len = len;
            buf ^= len & 1;
            q += len;
            rebuilt = 0;
        }
        ++A->nck;
    }
    // kept: the final history goes back into the live list, as the fused step leaves it
    if (A->keep && (rc = restore_from(A, s, live, A->traj[(size_t)S], false))) return rc;
    HIPCALL(c, launch_ctrl(c->d_flags, 3, S, c->stream));
    if ((rc = read_flags(c, h))) return rc;
    c->step_counter += S;
    c->binned = false;
    c->forces_valid = true;
    A->step_end = c->step_counter;
    return flag_error(c, h);
}

int dem_rollout_backward(dem_adjoint *A, const dem_state *s, const double *gx, const double *gv, const double *gw,
                         double *ax0, double *av0, double *aw0, int32_t *ids0, double *grad) {
    if (!A) return DEM_ERR_ARG;
    dem_ctx *c = A->ctx;
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!gx || !gv || !gw || !ax0 || !av0 || !aw0) return fail(c, DEM_ERR_ARG, "an adjoint array is NULL");
    if (c->fext_on) return fail(c, DEM_ERR_STATE, "the reverse mode does not take external forces");
    if (A->nck < 2 || A->step_end != c->step_counter)
        return fail(c, DEM_ERR_STATE, "dem_rollout_backward needs the state of the last dem_rollout_forward");
    const int64_t n = c->geo.n, K = A->kslots;
    const int nt = c->geo.sys[0].ntypes;
    hipStream_t st = c->stream;
    if ((rc = fill_zero(A, A->acc, (size_t)5 * nt * nt)) || (rc = fill_zero(A, A->gp, (size_t)5 * nt * n)) ||
        (rc = fill_zero(A, A->mu[0], (size_t)4 * n * K)) || (rc = fill_zero(A, A->muw[0], (size_t)4 * n)))
        return rc;
    const AArgs a0 = base_args(A);
    int cur = 0, m = 0;
    {
        AArgs a = a0;
        a.im = at<D2>(A, A->topo[A->ck[A->nck - 1].topo].im);
        a.rout = at<D4>(A, A->rec[0]);
        HIPCALL(c, launch_adj_seed(a, gx, gv, gw, st));
    }
    for (int w = A->nck - 1; w >= 1; --w) {
        const Ckpt &C = A->ck[w];
        const Topo &T = A->topo[C.topo];
        AArgs a = a0;
        a.nbr = at<int32_t>(A, T.nbr);
        a.cnt = at<int32_t>(A, T.cnt);
        a.im = at<D2>(A, T.im);
        a.gp = at<double>(A, A->gp);
        auto in_of = [&](int t, AArgs &x) {
            if (A->keep) {
                const StepBuf &B = A->traj[(size_t)(C.q0 + t) - 1];
                x.pos = at<D4>(A, B.pos); x.vel = at<D4>(A, B.vel); x.spin = at<D4>(A, B.spin);
                x.hin = at<D4>(A, B.hist); x.hwin = at<D4>(A, B.hw);
            } else if (t == 0) {
                x.pos = at<D4>(A, C.pos); x.vel = at<D4>(A, C.vel); x.spin = at<D4>(A, C.spin);
                x.hin = at<D4>(A, C.hist); x.hwin = at<D4>(A, C.hw);
            } else {
                const StepBuf &B = A->traj[t - 1];
                x.pos = at<D4>(A, B.pos); x.vel = at<D4>(A, B.vel); x.spin = at<D4>(A, B.spin);
                x.hin = at<D4>(A, B.hist); x.hwin = at<D4>(A, B.hw);
            }
        };
        for (int t = 0; !A->keep && t + 1 < C.len; ++t) {
            in_of(t, a);
            const StepBuf &B = A->traj[t];
            a.pos_o = at<D4>(A, B.pos); a.vel_o = at<D4>(A, B.vel); a.spin_o = at<D4>(A, B.spin);
            a.hout = at<D4>(A, B.hist); a.hwout = at<D4>(A, B.hw);
            HIPCALL(c, launch_adj_forward(a, 0, st));
        }
        a.mu = at<D4>(A, A->mu[m]);
        a.muw = at<D4>(A, A->muw[m]);
        for (int t = C.len - 1; t >= 0; --t) {
            in_of(t, a);
            a.rin = at<D4>(A, A->rec[cur]);
            a.rout = at<D4>(A, A->rec[cur ^ 1]);
            HIPCALL(c, launch_adj_reverse(a, 0, st));
            cur ^= 1;
        }
        in_of(0, a);
        HIPCALL(c, launch_adj_reduce(a, at<double>(A, A->part), at<double>(A, A->acc), st));
        if ((rc = fill_zero(A, A->gp, (size_t)5 * nt * n))) return rc;
        if (C.rebuilt) {
            const Topo &O = A->topo[A->ck[w - 1].topo];
            a.rin = at<D4>(A, A->rec[cur]);
            a.rout = at<D4>(A, A->rec[cur ^ 1]);
            HIPCALL(c, launch_adj_carry(a, at<int32_t>(A, T.frame), at<int32_t>(A, T.ids), at<int32_t>(A, O.nbr),
                                        at<int32_t>(A, O.cnt), at<int32_t>(A, O.ids), at<D4>(A, A->mu[m ^ 1]),
                                        at<D4>(A, A->muw[m ^ 1]), st));
            cur ^= 1;
            m ^= 1;
        }
    }
    {
        // the force evaluation before the first kick: history untouched, the
        // force enters u_1 through one half kick
        const Ckpt &C = A->ck[0];
        const Topo &T = A->topo[C.topo];
        AArgs a = a0;
        a.nbr = at<int32_t>(A, T.nbr);
        a.cnt = at<int32_t>(A, T.cnt);
        a.im = at<D2>(A, T.im);
        a.pos = at<D4>(A, C.pos); a.vel = at<D4>(A, C.vel); a.spin = at<D4>(A, C.spin);
        a.hin = at<D4>(A, C.hist); a.hwin = at<D4>(A, C.hw);
        a.rin = at<D4>(A, A->rec[cur]);
        a.mu = at<D4>(A, A->mu[m]);
        a.muw = at<D4>(A, A->muw[m]);
        a.gp = at<double>(A, A->gp);
        a.seed_scale = 0.5;
        a.ox = ax0; a.ov = av0; a.ow = aw0;
        HIPCALL(c, launch_adj_reverse(a, 1, st));
        HIPCALL(c, launch_adj_reduce(a, at<double>(A, A->part), at<double>(A, A->acc), st));
        if (ids0) HIPCALL(c, hipMemcpyAsync(ids0, A->ws + T.ids, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
    }
    return finish_grad(A, grad);
}

int dem_forces_vjp(dem_adjoint *A, const dem_state *s, const double *fb, const double *tb, double *xb, double *vb,
                   double *wb, double *grad) {
    if (!A) return DEM_ERR_ARG;
    dem_ctx *c = A->ctx;
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!fb || !tb || !xb || !vb || !wb) return fail(c, DEM_ERR_ARG, "an adjoint array is NULL");
    if (c->fext_on) return fail(c, DEM_ERR_STATE, "the reverse mode does not take external forces");
    if (c->geo.sys[0].pe != c->geo.sys[0].p1)
        return fail(c, DEM_ERR_STATE, "the reverse mode takes a system without free slots");
    if (!c->list_current) return fail(c, DEM_ERR_STATE, "dem_forces_vjp needs a neighbour list for the current order");
    if (c->geo.n == 0) return DEM_OK;
    const int64_t n = c->geo.n, K = A->kslots;
    const int nt = c->geo.sys[0].ntypes;
    hipStream_t st = c->stream;
    List live;
    if ((rc = live_list(c, 0, live)) || (rc = check_rows(A, live))) return rc;
    KArgs Kx = kargs(c, s);
    HIPCALL(c, launch_pack(Kx, 0, 0, 0, 0, st));
    const Ckpt &C = A->ck[0];
    AArgs a = base_args(A);
    a.nbr = live.nbr;
    a.cnt = live.cnt;
    a.im = Kx.im;
    a.pos = Kx.pos[0]; a.vel = Kx.vel[0]; a.spin = Kx.spin[0];
    HIPCALL(c, launch_adj_expand(a, live.xi, live.mask, Kx.xiw, at<D4>(A, C.hist), at<D4>(A, C.hw), st));
    a.hin = at<D4>(A, C.hist);
    a.hwin = at<D4>(A, C.hw);
    if ((rc = fill_zero(A, A->acc, (size_t)5 * nt * nt)) || (rc = fill_zero(A, A->gp, (size_t)5 * nt * n)) ||
        (rc = fill_zero(A, A->mu[0], (size_t)4 * n * K)) || (rc = fill_zero(A, A->muw[0], (size_t)4 * n)))
        return rc;
    a.rout = at<D4>(A, A->rec[0]);
    HIPCALL(c, launch_adj_seed_forces(a, fb, tb, st));
    a.rin = at<D4>(A, A->rec[0]);
    a.mu = at<D4>(A, A->mu[0]);
    a.muw = at<D4>(A, A->muw[0]);
    a.gp = at<double>(A, A->gp);
    a.seed_scale = 1.0;
    a.ox = xb; a.ov = vb; a.ow = wb;
    HIPCALL(c, launch_adj_reverse(a, 1, st));
    HIPCALL(c, launch_adj_reduce(a, at<double>(A, A->part), at<double>(A, A->acc), st));
    return finish_grad(A, grad);
}

int dem_integrate_vjp(dem_ctx *c, const dem_state *s, int32_t phase, const double *xb, const double *vb,
                      const double *wb, double *x_in, double *v_in, double *w_in, double *f_in, double *t_in) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (phase != 0 && phase != 1) return fail(c, DEM_ERR_ARG, "phase must be 0 or 1");
    if (c->geo.n > 0 && (!xb || !vb || !wb || !x_in || !v_in || !w_in || !f_in || !t_in))
        return fail(c, DEM_ERR_ARG, "an adjoint array is NULL");
    if (!c->masses) return fail(c, DEM_ERR_STATE, "dem_reset first (the masses)");
    const KArgs a = kargs(c, s);
    HIPCALL(c, launch_integrate_vjp(c->d_sys, (int)c->geo.sys.size(), c->geo.n, a.inv_m, a.inv_I, phase, xb, vb, wb,
                                    x_in, v_in, w_in, f_in, t_in, c->stream));
    return DEM_OK;
}

int dem_adjoint_set_lanes(dem_adjoint *A, int32_t lanes) {
    if (!A) return DEM_ERR_ARG;
    if (lanes != 4 && lanes != 8) return fail(A->ctx, DEM_ERR_ARG, "lanes must be 4 or 8");
    A->lanes = lanes;
    return DEM_OK;
}

int dem_adjoint_info(dem_adjoint *A, int64_t out[4]) {
    if (!A || !out) return DEM_ERR_ARG;
    out[0] = A->nck > 0 ? A->nck - 1 : 0;
    out[1] = A->rebuilds;
    out[2] = (int64_t)A->bytes;
    out[3] = A->max_windows;
    return DEM_OK;
}

int dem_adjoint_destroy(dem_adjoint *A) {
    delete A;
    return DEM_OK;
}

}  // extern "C"
