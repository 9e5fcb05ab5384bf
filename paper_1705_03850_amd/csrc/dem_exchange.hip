// dem_exchange.hip -- insertion and deletion of spheres at the boundary of the
// fine region of the multi-level coarse-grain model (Sec. 2.3): the C-ABI
// calls dem_exchange and dem_live_count and their kernels.
//
// One event on one system, all on the device:
//   budget     one thread per boundary cell: the carried budget plus the
//              inflow of the interval (into a scratch copy);
//   mark       one thread per live sphere of the context: the largest id,
//              and for the system the removal marks (half-space test) and the
//              identity frame (each kept sphere's previous list row is its
//              own);
//   candidates one thread per candidate: validation, its mass, its cell of
//              the system's binning grid; a counting sort of the candidates
//              by that cell;
//   existing   one thread per candidate: any overlap with a kept sphere, over
//              the 27 cells around it (spheres stay within skin/2 of their
//              binned position, so an overlapping sphere is binned in one of
//              them);
//   conflicts  one thread per candidate: the earlier candidates (not blocked
//              by a kept sphere) that it overlaps, from the 27 cells of the
//              candidates' own binning;
//   SSI        one wave walks the candidates in order (their data read 64 at
//              a time and broadcast from the lane that holds it): budget test,
//              conflicts against the accepted ones (lanes split the list, a
//              ballot decides), budget charged -- the only sequential part;
//   insert     one thread per accepted candidate, written after the live
//              spheres; then the list rebuild of the system, whose binning
//              sends removed spheres to the spare cell past the grid (so
//              the live ones end up first) and carries every kept pair's
//              history by id, and the system's force pass at the new state
//              (history untouched; the other systems are not touched).
// Nothing the caller sees changes before the acceptance is known to fit:
// budget and accepted flags live in scratch until then.
#include <cmath>
#include <cstring>

#include "dem_ctx.h"

namespace dem {
namespace {

constexpr int kConf = 32;                 // earlier overlapping candidates kept per candidate
constexpr int64_t kMaxCand = 1 << 18;     // candidates per call (acceptance bits in LDS)

enum : int { kExBadCandidate = 1, kExConflicts = 2, kExStale = 4 };

struct ExArgs {
    int32_t sys;
    int64_t K;                 // candidates
    const double *cx;          // [3][K]
    const double *cr;          // [K]
    const int32_t *ct, *cc;    // [K] type, boundary cell
    const double *fields;      // [DEM_NFIELDS][nb]
    const double *budget_in;   // [nb]
    int64_t nb;                // boundary cells
    double nrm[3], face, slab, interval;
    double onrm[3], oface;     // outlet half-space (onrm = 0: none)
    int32_t outlet;
    // scratch (in the binning scratch, free between list builds)
    int32_t *blocked;   // [K] 1: overlaps a kept sphere
    double *mass;       // [K]
    int32_t *ccell;     // [K] cell of the system's grid
    int32_t *crank;     // [K] rank within that cell
    int32_t *corder;    // [K] candidates ordered by cell
    int32_t *nconf;     // [K]
    int32_t *conf;      // [K][kConf] earlier overlapping candidates
    int32_t *acc;       // [K] accepted flags
    int32_t *alist;     // [K] accepted candidates in order
    double *bud;        // [nb] budget
    int32_t *ccount;    // [ncs] candidates per cell
    int32_t *cstart;    // [ncs + 1] exclusive scan of ccount
    int32_t *cpart;     // scan partials
    int64_t ncs;        // cells of the system's grid
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane j's value of v (j the same in every lane).
__device__ __forceinline__ double readlane_f64(double v, int j) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, j);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), j);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Squared distance of two centres, the minimum image on periodic axes, in the
// order (dx dx + dy dy) + dz dz.
__device__ __forceinline__ double dist2(const SysDesc &s, double ax, double ay, double az, double bx, double by,
                                        double bz) {
    const double dx = min_image(ax - bx, s.L[0], s.hL[0], s.periodic[0]);
    const double dy = min_image(ay - by, s.L[1], s.hL[1], s.periodic[1]);
    const double dz = min_image(az - bz, s.L[2], s.hL[2], s.periodic[2]);
    return dx * dx + dy * dy + dz * dz;
}

// The distinct cells around (cx, cy, cz) of the system's grid (periodic axes
// wrap; open axes stop at the grid).
template <class F>
__device__ inline void for_adjacent_cells(const SysDesc &s, int cx, int cy, int cz, F visit) {
    for (int dz = -1; dz <= 1; ++dz) {
        int z = cz + dz;
        if (s.periodic[2]) {
            if (s.nc[2] < 3 && dz == -1) continue;
            z = z < 0 ? z + s.nc[2] : (z >= s.nc[2] ? z - s.nc[2] : z);
        } else if (z < 0 || z >= s.nc[2]) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            int y = cy + dy;
            if (s.periodic[1]) {
                if (s.nc[1] < 3 && dy == -1) continue;
                y = y < 0 ? y + s.nc[1] : (y >= s.nc[1] ? y - s.nc[1] : y);
            } else if (y < 0 || y >= s.nc[1]) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                int x = cx + dx;
                if (s.periodic[0]) {
                    if (s.nc[0] < 3 && dx == -1) continue;
                    x = x < 0 ? x + s.nc[0] : (x >= s.nc[0] ? x - s.nc[0] : x);
                } else if (x < 0 || x >= s.nc[0]) continue;
                visit(((int64_t)z * s.nc[1] + y) * s.nc[0] + x);
            }
        }
    }
}

__global__ void k_ex_budget(ExArgs e) {
    const double *P = e.fields + (int64_t)DEM_F_MOM * e.nb;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < e.nb; c += (int64_t)gridDim.x * blockDim.x) {
        double b = e.budget_in[c];
        if (e.interval > 0.0) {
            const double flow = P[c] * e.nrm[0] + P[e.nb + c] * e.nrm[1] + P[2 * e.nb + c] * e.nrm[2];
            b = b + fmax(flow, 0.0) / e.slab * e.interval;
        }
        e.bud[c] = b;
    }
}

// Largest live id of the context; removal marks, identity frames and the list
// validity check for the system.
__global__ void k_ex_mark(KArgs a, ExArgs e) {
    const int64_t n = a.n;
    const SysDesc &s = a.sys[e.sys];
    int32_t mx = -1;
    int removed = 0, stale = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = a.nsys - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (i < a.sys[mid].p1) hi = mid;
            else lo = mid + 1;
        }
        if (i >= a.sys[lo].pe) continue;   // a free slot
        mx = max(mx, a.id[i]);
        if (lo != e.sys) continue;
        const double x = a.x[i], y = a.x[n + i], z = a.x[2 * n + i];
        int out = (x * e.nrm[0] + y * e.nrm[1] + z * e.nrm[2]) < e.face ? 1 : 0;
        if (e.outlet && (x * e.onrm[0] + y * e.onrm[1] + z * e.onrm[2]) < e.oface) out = 1;
        a.dead[i] = out;
        a.frame[i] = (int32_t)i;
        removed += out;
        // an overlapping sphere must be binned next to the candidate's cell
        for (int ax = 0; ax < 3; ++ax)
            if (!(fabs(a.disp[ax * n + i]) <= 1.0 / s.inv_w[ax] - 2.0 * s.rmax)) stale = 1;
    }
    for (int off = warpSize / 2; off > 0; off >>= 1) {
        mx = max(mx, __shfl_xor(mx, off));
        removed += __shfl_xor(removed, off);
        stale |= __shfl_xor(stale, off);
    }
    if ((threadIdx.x % warpSize) == 0) {
        if (mx >= 0) atomicMax(&a.flags->ex_maxid, mx);
        if (removed) atomicAdd((unsigned long long *)&a.flags->ex_removed, (unsigned long long)removed);
        if (stale) atomicOr(&a.flags->ex_err, kExStale);
    }
}

__global__ void k_ex_candidates(KArgs a, ExArgs e) {
    const SysDesc &s = a.sys[e.sys];
    const int64_t K = e.K;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const double x[3] = {e.cx[k], e.cx[K + k], e.cx[2 * K + k]};
        const double r = e.cr[k];
        const int t = e.ct[k];
        const int cb = e.cc[k];
        bool ok = t >= 0 && t < s.ntypes && r > 0.0 && r <= s.rmax && cb >= 0 && cb < e.nb;
        for (int ax = 0; ax < 3; ++ax) {
            if (!isfinite(x[ax])) ok = false;
            else if (s.periodic[ax] && !(x[ax] >= s.lo[ax] && x[ax] < s.hi[ax])) ok = false;
        }
        if (!ok) {
            atomicOr(&a.flags->ex_err, kExBadCandidate);
            e.ccell[k] = 0;
            e.mass[k] = 0.0;
            e.crank[k] = atomicAdd(&e.ccount[0], 1);
            continue;
        }
        const double rho = a.rho[s.type0 + t];
        e.mass[k] = 4.0 / 3.0 * M_PI * rho * r * r * r;
        const int cx = cell_coord(x[0], s, 0), cy = cell_coord(x[1], s, 1), cz = cell_coord(x[2], s, 2);
        const int32_t c = (int32_t)(((int64_t)cz * s.nc[1] + cy) * s.nc[0] + cx);
        e.ccell[k] = c;
        e.crank[k] = atomicAdd(&e.ccount[c], 1);
    }
}

__global__ void k_ex_place(ExArgs e) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < e.K; k += (int64_t)gridDim.x * blockDim.x)
        e.corder[e.cstart[e.ccell[k]] + e.crank[k]] = (int32_t)k;
}

// Candidate k against the kept spheres binned around it.
__global__ void k_ex_existing(KArgs a, ExArgs e) {
    const SysDesc &s = a.sys[e.sys];
    const int64_t n = a.n, K = e.K;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const double xk = e.cx[k], yk = e.cx[K + k], zk = e.cx[2 * K + k], rk = e.cr[k];
        const int cx = cell_coord(xk, s, 0), cy = cell_coord(yk, s, 1), cz = cell_coord(zk, s, 2);
        int hit = 0;
        for_adjacent_cells(s, cx, cy, cz, [&](int64_t c) {
            if (hit) return;
            const int32_t b = a.cell_start[s.c0 + c], end = a.cell_start[s.c0 + c + 1];
            for (int32_t j = b; j < end; ++j) {
                if (a.dead[j]) continue;
                const double d2 = dist2(s, xk, yk, zk, a.x[j], a.x[n + j], a.x[2 * n + j]);
                const double sr = rk + a.r[j];
                if (d2 < sr * sr) {
                    hit = 1;
                    break;
                }
            }
        });
        e.blocked[k] = hit;
    }
}

// Earlier candidates (not blocked) that candidate k overlaps.
__global__ void k_ex_conflicts(KArgs a, ExArgs e) {
    const SysDesc &s = a.sys[e.sys];
    const int64_t K = e.K;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        int cnt = 0;
        if (!e.blocked[k]) {
            const double xk = e.cx[k], yk = e.cx[K + k], zk = e.cx[2 * K + k], rk = e.cr[k];
            const int cx = cell_coord(xk, s, 0), cy = cell_coord(yk, s, 1), cz = cell_coord(zk, s, 2);
            for_adjacent_cells(s, cx, cy, cz, [&](int64_t c) {
                for (int32_t p = e.cstart[c]; p < e.cstart[c + 1]; ++p) {
                    const int32_t j = e.corder[p];
                    if (j >= k || e.blocked[j]) continue;
                    const double d2 = dist2(s, xk, yk, zk, e.cx[j], e.cx[K + j], e.cx[2 * K + j]);
                    const double sr = rk + e.cr[j];
                    if (d2 < sr * sr) {
                        if (cnt < kConf) e.conf[k * kConf + cnt] = j;
                        ++cnt;
                    }
                }
            });
            if (cnt > kConf) atomicOr(&a.flags->ex_err, kExConflicts);
        }
        e.nconf[k] = cnt < kConf ? cnt : kConf;
    }
}

// The sequential acceptance, one wave: candidates in order, 64 at a time.
__global__ void __launch_bounds__(64) k_ex_ssi(ExArgs e, Flags *flags) {
    __shared__ uint32_t bits[kMaxCand / 32];   // accepted flags
    const int lane = threadIdx.x;
    const int64_t K = e.K;
    for (int64_t w = lane; w < (K + 31) / 32; w += 64) bits[w] = 0;
    wave_sync();
    int64_t nacc = 0;
    for (int64_t base = 0; base < K; base += 64) {
        const int64_t mine = base + lane;
        int b = 1, cb = 0, nc = 0;
        double m = 0.0;
        if (mine < K) {
            b = e.blocked[mine];
            cb = e.cc[mine];
            nc = e.nconf[mine];
            m = e.mass[mine];
        }
        const int len = K - base < 64 ? (int)(K - base) : 64;
        for (int j = 0; j < len; ++j) {
            const int64_t k = base + j;
            if (__builtin_amdgcn_readlane(b, j)) continue;
            const int c = __builtin_amdgcn_readlane(cb, j);
            if (c < 0 || c >= e.nb) continue;   // a bad candidate (the call then fails)
            const double mk = readlane_f64(m, j);
            const double left = e.bud[c];
            if (!(mk <= left)) continue;
            const int ncf = __builtin_amdgcn_readlane(nc, j);
            int clash = 0;
            if (lane < ncf) {
                const int32_t q = e.conf[k * kConf + lane];
                clash = (bits[q >> 5] >> (q & 31)) & 1;
            }
            if (__ballot(clash)) continue;
            // accepted: every lane stores the same values
            e.bud[c] = left - mk;
            if (lane == 0) {
                bits[k >> 5] |= 1u << (k & 31);
                e.alist[nacc] = (int32_t)k;
            }
            wave_sync();
            ++nacc;
        }
    }
    wave_sync();
    for (int64_t k = lane; k < K; k += 64) e.acc[k] = (bits[k >> 5] >> (k & 31)) & 1;
    if (lane == 0) flags->ex_accepted = nacc;
}

// Accepted candidate q becomes particle pe + q of the system.
__global__ void k_ex_insert(KArgs a, ExArgs e, int64_t pe, int64_t nacc, int32_t id0) {
    const SysDesc &s = a.sys[e.sys];
    const int64_t n = a.n, K = e.K, nb = e.nb;
    const double *M = e.fields + (int64_t)DEM_F_MASS * nb;
    const double *P = e.fields + (int64_t)DEM_F_MOM * nb;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nacc; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e.alist[q];
        const int64_t i = pe + q;
        const int cb = e.cc[k];
        const double mc = M[cb];
        for (int ax = 0; ax < 3; ++ax) {
            a.x[ax * n + i] = e.cx[ax * K + k];
            a.v[ax * n + i] = mc > 0.0 ? P[ax * nb + cb] / mc : 0.0;   // the cell's Favre velocity
            a.w[ax * n + i] = 0.0;
            a.f[ax * n + i] = 0.0;
            a.t[ax * n + i] = 0.0;
            a.disp[ax * n + i] = 0.0;
            a.xiw[ax * n + i] = 0.0;
            a.fext_ws[ax * n + i] = 0.0;
        }
        const double r = e.cr[k];
        const int t = e.ct[k];
        a.r[i] = r;
        a.type[i] = t;
        a.id[i] = id0 + (int32_t)q;
        a.frame[i] = -1;   // no row in the previous list
        a.dead[i] = 0;
        if (a.smask) a.smask[i] = 0;
        const double rho = a.rho[s.type0 + t];
        const double m = 4.0 / 3.0 * M_PI * rho * r * r * r;
        const double I = 0.4 * m * r * r;
        a.m[i] = m;
        a.inv_m[i] = 1.0 / m;
        a.inv_I[i] = 1.0 / I;
    }
}

__global__ void k_ex_out(ExArgs e, double *budget, int32_t *accepted) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < e.nb; c += stride) budget[c] = e.bud[c];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < e.K; k += stride) accepted[k] = e.acc[k];
}

__global__ void k_ex_clear(KArgs a, int32_t sys) {
    const SysDesc &s = a.sys[sys];
    for (int64_t i = s.p0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s.p1;
         i += (int64_t)gridDim.x * blockDim.x)
        a.dead[i] = 0;
}

__global__ void k_ex_reset(Flags *f) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        f->ex_removed = 0;
        f->ex_accepted = 0;
        f->ex_maxid = -1;
        f->ex_err = 0;
    }
}

__global__ void k_set_live_end(SysDesc *sys, int32_t s, int64_t pe) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sys[s].pe = pe;
}

int blocks_for(int64_t work, int block) {
    int64_t b = (work + block - 1) / block;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace
}  // namespace dem

using namespace dem;
using namespace dem::host;

extern "C" {

int dem_live_count(dem_ctx *c, int32_t sys, int64_t *n) {
    if (!c || !n) return DEM_ERR_ARG;
    if (sys < 0 || sys >= (int32_t)c->geo.sys.size()) return fail(c, DEM_ERR_ARG, "sys out of range");
    *n = c->geo.sys[sys].pe - c->geo.sys[sys].p0;
    return DEM_OK;
}

int dem_exchange(dem_ctx *c, const dem_state *s, int32_t sys, const dem_exchange_params *p, const double *fields,
                 double *budget, int64_t ncand, const double *cand_x, const double *cand_r, const int32_t *cand_type,
                 const int32_t *cand_cell, int32_t *accepted, int64_t counts[3]) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!p || !counts) return fail(c, DEM_ERR_ARG, "params or counts is NULL");
    if (sys < 0 || sys >= (int32_t)c->geo.sys.size()) return fail(c, DEM_ERR_ARG, "sys out of range");
    if (ncand < 0 || ncand > kMaxCand) return fail(c, DEM_ERR_ARG, "ncand must be in 0..262144");
    if (p->ncell < 1 || p->ncell > (1 << 24)) return fail(c, DEM_ERR_ARG, "ncell must be in 1..2^24");
    if (!fields || !budget) return fail(c, DEM_ERR_ARG, "fields or budget is NULL");
    if (ncand > 0 && (!cand_x || !cand_r || !cand_type || !cand_cell || !accepted))
        return fail(c, DEM_ERR_ARG, "a candidate array is NULL");
    const double nn = p->nrm[0] * p->nrm[0] + p->nrm[1] * p->nrm[1] + p->nrm[2] * p->nrm[2];
    if (!(std::fabs(nn - 1.0) < 1e-12)) return fail(c, DEM_ERR_ARG, "nrm must be a unit vector");
    const double on = p->out_nrm[0] * p->out_nrm[0] + p->out_nrm[1] * p->out_nrm[1] + p->out_nrm[2] * p->out_nrm[2];
    if (on != 0.0 && (!(std::fabs(on - 1.0) < 1e-12) || !std::isfinite(p->out_face)))
        return fail(c, DEM_ERR_ARG, "out_nrm must be zero or a unit vector (with a finite out_face)");
    if (!std::isfinite(p->face) || !(p->interval >= 0.0) || !std::isfinite(p->interval) ||
        (p->interval > 0.0 && !(p->slab > 0.0 && std::isfinite(p->slab))))
        return fail(c, DEM_ERR_ARG, "need a finite face, interval >= 0 and slab > 0 with an interval");
    if (!c->forces_valid || !c->list_current)
        return fail(c, DEM_ERR_STATE, "dem_exchange needs the forces of the current state (and its list)");
    SysDesc &sd = c->geo.sys[sys];
    const int64_t ncs = (int64_t)sd.nc[0] * sd.nc[1] * sd.nc[2];
    // scratch in the binning scratch (free until the list rebuild below)
    const int64_t K = ncand;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
    const size_t o_blocked = take(K * 4), o_mass = take(K * 8), o_ccell = take(K * 4), o_crank = take(K * 4),
                 o_corder = take(K * 4), o_nconf = take(K * 4), o_conf = take(K * kConf * 4), o_acc = take(K * 4),
                 o_alist = take(K * 4), o_bud = take(p->ncell * 8), o_ccount = take(ncs * 4),
                 o_cstart = take((ncs + 1) * 4), o_cpart = take(((ncs + 1023) / 1024 + 1) * 4);
    const size_t shadow_bytes = (size_t)kShadowD * c->geo.n * 8;
    if (off > shadow_bytes) return fail(c, DEM_ERR_CAPACITY, "too many candidates for the workspace's scratch");
    char *sc = c->ws + c->lay.shadow_d;
    ExArgs e;
    memset(&e, 0, sizeof e);
    e.sys = sys;
    e.K = K;
    e.cx = cand_x; e.cr = cand_r; e.ct = cand_type; e.cc = cand_cell;
    e.fields = fields;
    e.budget_in = budget;
    e.nb = p->ncell;
    for (int a = 0; a < 3; ++a) e.nrm[a] = p->nrm[a];
    e.face = p->face;
    for (int a = 0; a < 3; ++a) e.onrm[a] = p->out_nrm[a];
    e.oface = p->out_face;
    e.outlet = (p->out_nrm[0] != 0.0 || p->out_nrm[1] != 0.0 || p->out_nrm[2] != 0.0) ? 1 : 0;
    e.slab = p->slab;
    e.interval = p->interval;
    e.blocked = (int32_t *)(sc + o_blocked);
    e.mass = (double *)(sc + o_mass);
    e.ccell = (int32_t *)(sc + o_ccell);
    e.crank = (int32_t *)(sc + o_crank);
    e.corder = (int32_t *)(sc + o_corder);
    e.nconf = (int32_t *)(sc + o_nconf);
    e.conf = (int32_t *)(sc + o_conf);
    e.acc = (int32_t *)(sc + o_acc);
    e.alist = (int32_t *)(sc + o_alist);
    e.bud = (double *)(sc + o_bud);
    e.ccount = (int32_t *)(sc + o_ccount);
    e.cstart = (int32_t *)(sc + o_cstart);
    e.cpart = (int32_t *)(sc + o_cpart);
    e.ncs = ncs;
    KArgs a = kargs(c, s);
    hipStream_t st = c->stream;
    HIPCALL(c, hipGetLastError());
    k_ex_reset<<<1, 64, 0, st>>>(c->d_flags);
    k_ex_budget<<<blocks_for(e.nb, 256), 256, 0, st>>>(e);
    k_ex_mark<<<blocks_for(c->geo.n, 256), 256, 0, st>>>(a, e);
    if (K > 0) {
        HIPCALL(c, launch_fill_i32(e.ccount, ncs, 0, st));
        k_ex_candidates<<<blocks_for(K, 256), 256, 0, st>>>(a, e);
        HIPCALL(c, launch_scan(e.ccount, ncs, e.cpart, e.cstart, st));   // cstart[0..ncs]
        k_ex_place<<<blocks_for(K, 256), 256, 0, st>>>(e);
        k_ex_existing<<<blocks_for(K, 64), 64, 0, st>>>(a, e);
        k_ex_conflicts<<<blocks_for(K, 64), 64, 0, st>>>(a, e);
        k_ex_ssi<<<1, 64, 0, st>>>(e, c->d_flags);
    }
    HIPCALL(c, hipGetLastError());
    Flags h;
    if ((rc = read_flags(c, h))) return rc;
    const int64_t nacc = h.ex_accepted, nrem = h.ex_removed;
    std::string why;
    int code = DEM_OK;
    if (h.ex_err & kExBadCandidate) {
        code = DEM_ERR_ARG;
        why = "a candidate has a type out of range, r outside (0, r_max], a cell outside [0, ncell), a non-finite "
              "position or one outside the box on a periodic axis";
    } else if (h.ex_err & kExStale) {
        code = DEM_ERR_STATE;
        why = "a sphere moved too far from its binned position: the list does not match the positions";
    } else if (h.ex_err & kExConflicts) {
        code = DEM_ERR_CAPACITY;
        why = "a candidate overlaps more than 32 earlier candidates: pass fewer per call";
    } else if (sd.pe + nacc > sd.p1) {
        code = DEM_ERR_CAPACITY;
        why = "the accepted candidates do not fit the system's free slots (n_max)";
    } else if ((int64_t)h.ex_maxid + nacc > (int64_t)INT32_MAX) {
        code = DEM_ERR_CAPACITY;
        why = "new ids would pass 2^31 - 1";
    }
    if (code != DEM_OK) {
        k_ex_clear<<<blocks_for(sd.p1 - sd.p0, 256), 256, 0, st>>>(a, sys);
        HIPCALL(c, hipStreamSynchronize(st));
        return fail(c, code, why);
    }
    // ---- commit: outputs, new particles, then the system's list rebuild
    if (K > 0 || e.nb > 0) k_ex_out<<<blocks_for(std::max<int64_t>(K, e.nb), 256), 256, 0, st>>>(e, budget, accepted);
    if (nacc == 0 && nrem == 0) {   // nothing inserted or removed: list and forces stay valid
        HIPCALL(c, hipGetLastError());
        counts[0] = 0;
        counts[1] = 0;
        counts[2] = sd.pe - sd.p0;
        HIPCALL(c, hipStreamSynchronize(st));
        return DEM_OK;
    }
    const int64_t pe0 = sd.pe;
    if (nacc > 0) {
        k_ex_insert<<<blocks_for(nacc, 256), 256, 0, st>>>(a, e, pe0, nacc, h.ex_maxid + 1);
        k_set_live_end<<<1, 64, 0, st>>>(c->d_sys, sys, pe0 + nacc);
    }
    HIPCALL(c, hipGetLastError());
    HIPCALL(c, launch_fill_i32(a.sel, (int64_t)c->geo.sys.size(), 0, st));
    HIPCALL(c, launch_fill_i32(a.sel + sys, 1, 1, st));
    const bool win_was = c->win_on;
    int64_t win_old[4];
    memcpy(win_old, c->win, sizeof win_old);
    c->win[0] = sd.p0;
    c->win[1] = sd.p1;
    c->win[2] = sd.c0;
    c->win[3] = sd.c0 + ncs + 1;
    c->win_on = true;
    a = kargs(c, s);
    hipError_t he = launch_bin(a, 0, st);   // previous rows from the frames set above
    const int64_t pe1 = pe0 + nacc - nrem;
    if (he == hipSuccess) {
        k_set_live_end<<<1, 64, 0, st>>>(c->d_sys, sys, pe1);
        he = hipGetLastError();
    }
    if (he == hipSuccess) he = launch_neighbors(a, 1, st);
    if (he == hipSuccess) he = launch_flip(a, st);
    if (he == hipSuccess) he = launch_fill_i32(a.sel, (int64_t)c->geo.sys.size(), 0, st);
    if (he == hipSuccess) he = launch_ctrl(c->d_flags, 4, 1, st);
    c->win_on = win_was;
    memcpy(c->win, win_old, sizeof win_old);
    if (he != hipSuccess) return hip_fail(c, he, "list rebuild after the exchange");
    sd.pe = pe1;
    if ((rc = upload_tiles(c))) return rc;   // the step's tiles follow the live count
    // the system's forces at its new state, history untouched (the other
    // systems' forces stay as they are)
    if (he == hipSuccess) {
        KArgs af = kargs(c, s);
        af.only_sys = sys;
        he = launch_pack(af, 0, 0, 0, 0, st);
        if (he == hipSuccess) he = launch_step(af, 0, 0, 0, 0, 0, st);
    }
    if (he != hipSuccess) return hip_fail(c, he, "force pass after the exchange");
    c->have_list = true;
    c->list_current = true;
    c->binned = true;
    c->frame_identity = true;
    c->forces_valid = true;
    c->step_counter += 1;      // a reverse-mode trajectory recorded before no longer matches
    counts[0] = nacc;
    counts[1] = nrem;
    counts[2] = pe1 - sd.p0;
    if ((rc = read_flags(c, h))) return rc;
    return flag_error(c, h);
}

}  // extern "C"
