// dem_kernels.hip -- gfx950 kernels of the DEM contact pipeline.
//
//   binning           counting sort of particles by cell (cell major, id minor)
//   neighbour list    full directed rows sorted by neighbour id, history carried by id
//   forces            per-particle gather over its own row (Eq. (3)-(6), gravity, wall);
//                     no atomics in the force sums, fixed summation order
//   integration       velocity Verlet halves for Eq. (1)-(2)
//
// Every particle kernel walks tiles of `blockDim.x` particles.  Tiles are
// split into 8 contiguous chunks, one per XCD (workgroups are dispatched to
// the XCDs round-robin), so that a particle's neighbours -- close in the cell
// order -- are mostly read through the same L2.
#include "dem_kernels.h"

#include <float.h>

namespace dem {

constexpr int kXcd = 8;

struct TileIter {
    int64_t t, tend, stride;
};

__device__ inline TileIter tiles(int64_t n) {
    int64_t ntiles = (n + blockDim.x - 1) / blockDim.x;
    int per = gridDim.x / kXcd;
    int xcd = blockIdx.x % kXcd;
    int q = blockIdx.x / kXcd;
    int64_t chunk = (ntiles + kXcd - 1) / kXcd;
    int64_t t0 = xcd * chunk;
    int64_t t1 = t0 + chunk < ntiles ? t0 + chunk : ntiles;
    return TileIter{t0 + q, t1, per};
}

#define FOR_EACH_PARTICLE(n, i)                                                  \
    for (TileIter _it = tiles(n); _it.t < _it.tend; _it.t += _it.stride)         \
        for (int64_t i = _it.t * blockDim.x + threadIdx.x; i < (n); i = (n))

template <bool BATCH>
__device__ inline int sys_of(const KArgs &a, int64_t i) {
    if (!BATCH) return 0;
    int lo = 0, hi = a.nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (i < a.sys[mid].p1) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ inline double wrap_axis(double x, const SysDesc &s, int ax) {
    if (!s.periodic[ax]) return x;
    if (x >= s.hi[ax]) x -= s.L[ax];
    if (x < s.lo[ax]) x += s.L[ax];
    if (x >= s.hi[ax]) x = s.lo[ax];
    return x;
}

// ------------------------------------------------------------------ utilities

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f64(double *p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// op 0: clear abort, set step_base = value; op 1: step_base += value;
// op 2: clear the flag block (errors, counters); op 3: steps += value;
// op 4: builds += value
__global__ void k_ctrl(Flags *f, int op, int64_t value) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    if (op == 0) { f->abort_at = INT64_MAX; f->step_base = value; }
    else if (op == 1) { f->step_base += value; }
    else if (op == 2) {
        f->err = 0; f->max_row = 0; f->abort_at = INT64_MAX; f->step_base = 0;
        f->steps = 0; f->builds = 0; f->contacts = 0; f->wall_contacts = 0;
    } else if (op == 3) { f->steps += value; }
    else if (op == 4) { f->builds += value; }
}

// ------------------------------------------------------------------ masses

// Also validates what later kernels index with: type in [0, ntypes), id >= 0,
// r > 0 (a bad particle is flagged and its type forced to 0).
template <bool BATCH>
__global__ void k_init_mass(KArgs a) {
    bool bad = false;
    FOR_EACH_PARTICLE(a.n, i) {
        const SysDesc &s = a.sys[sys_of<BATCH>(a, i)];
        double r = a.r[i];
        int ty = a.type[i];
        if (ty < 0 || ty >= s.ntypes || a.id[i] < 0 || !(r > 0.0) || !isfinite(r)) {
            bad = true;
            ty = 0;
            a.type[i] = 0;
        }
        double rho = a.rho[s.type0 + ty];
        double m = 4.0 / 3.0 * M_PI * rho * r * r * r;
        double I = 0.4 * m * r * r;
        a.m[i] = m;
        a.inv_m[i] = 1.0 / m;
        a.inv_I[i] = 1.0 / I;
    }
    if (bad) atomicOr(&a.flags->err, kErrBadInput);
}

// ------------------------------------------------------------- integration

// Phase 0 of velocity Verlet: kick 1/2, drift, wrap, displacement since the
// last list build.  With gate != 0 the kernel belongs to step
// step_base + k of a chunk and does nothing once an earlier step of the chunk
// asked for a rebuild; it asks for one itself when a particle has moved more
// than skin/2.
template <bool BATCH>
__global__ void k_phase0(KArgs a, int k, int gate) {
    int64_t step = 0;
    if (gate) {
        step = a.flags->step_base + k;
        if (a.flags->abort_at < step) return;
    }
    bool need = false, bad = false;
    const int64_t n = a.n;
    FOR_EACH_PARTICLE(n, i) {
        const SysDesc &s = a.sys[sys_of<BATCH>(a, i)];
        double im = a.inv_m[i], iI = a.inv_I[i];
        double p[3], dsq = 0.0;
        for (int c = 0; c < 3; ++c) {
            double v = a.v[c * n + i] + s.hdt * (a.f[c * n + i] * im);
            double w = a.w[c * n + i] + s.hdt * (a.t[c * n + i] * iI);
            double x = a.x[c * n + i] + s.dt * v;
            x = wrap_axis(x, s, c);
            double d = a.disp[c * n + i] + s.dt * v;
            a.v[c * n + i] = v;
            a.w[c * n + i] = w;
            a.x[c * n + i] = x;
            a.disp[c * n + i] = d;
            dsq += d * d;
            p[c] = x + v;
        }
        if (!(dsq <= s.disp_thr2)) need = true;  // also true for NaN
        if (!isfinite(p[0] + p[1] + p[2])) bad = true;
    }
    if (bad) atomicOr(&a.flags->err, kErrNonFinite);
    if (need && gate) a.flags->abort_at = step;
}

// Phase 1: kick 1/2 with the new forces.
template <bool BATCH>
__global__ void k_phase1(KArgs a, int k, int gate) {
    if (gate) {
        int64_t step = a.flags->step_base + k;
        if (a.flags->abort_at <= step) return;
        if (blockIdx.x == 0 && threadIdx.x == 0) a.flags->steps += 1;
    }
    const int64_t n = a.n;
    FOR_EACH_PARTICLE(n, i) {
        const SysDesc &s = a.sys[sys_of<BATCH>(a, i)];
        double im = a.inv_m[i], iI = a.inv_I[i];
        for (int c = 0; c < 3; ++c) {
            a.v[c * n + i] = a.v[c * n + i] + s.hdt * (a.f[c * n + i] * im);
            a.w[c * n + i] = a.w[c * n + i] + s.hdt * (a.t[c * n + i] * iI);
        }
    }
}

// ------------------------------------------------------------------ forces

// One thread per particle: gravity, then every slot of its row (ascending
// neighbour id), then the wall.  Pair terms are evaluated from this
// particle's side only; the partner evaluates the mirrored contact in its own
// row, which gives the exact negative (see contact_force).  With update the
// slot history is advanced and stored; slots that are out of contact simply
// lose their mask bit (their history reads as zero from then on).
template <bool BATCH, bool COUNT>
__global__ void __launch_bounds__(256) k_forces(KArgs a, int update, int k, int gate) {
    if (gate) {
        int64_t step = a.flags->step_base + k;
        if (a.flags->abort_at <= step) return;
    }
    const int64_t n = a.n;
    const List L = a.cur;
    unsigned ncont = 0, nwall = 0;
    FOR_EACH_PARTICLE(n, i) {
        const SysDesc &s = a.sys[sys_of<BATCH>(a, i)];
        const PairCoef *coef = a.coef + s.coef0;
        const double xi = a.x[i], yi = a.x[n + i], zi = a.x[2 * n + i];
        const double vxi = a.v[i], vyi = a.v[n + i], vzi = a.v[2 * n + i];
        const double wxi = a.w[i], wyi = a.w[n + i], wzi = a.w[2 * n + i];
        const double ri = a.r[i], mi = a.m[i];
        const int ti = a.type[i];
        double Fx = mi * s.g[0], Fy = mi * s.g[1], Fz = mi * s.g[2];
        double Tx = 0.0, Ty = 0.0, Tz = 0.0;
        const int cnt = L.cnt[i];
        const uint64_t mask = L.mask[i];
        uint64_t nmask = 0;
        for (int q = 0; q < cnt; ++q) {
            const int32_t j = L.nbr[(int64_t)q * n + i];
            ContactIn c;
            c.dx = min_image(xi - a.x[j], s.L[0], s.hL[0], s.periodic[0]);
            c.dy = min_image(yi - a.x[n + j], s.L[1], s.hL[1], s.periodic[1]);
            c.dz = min_image(zi - a.x[2 * n + j], s.L[2], s.hL[2], s.periodic[2]);
            c.ra = ri;
            c.rb = a.r[j];
            const double d2 = c.dx * c.dx + c.dy * c.dy + c.dz * c.dz;
            const double rs = c.ra + c.rb;
            if (!(d2 < rs * rs)) continue;
            c.ma = mi;
            c.mb = a.m[j];
            c.vrx = vxi - a.v[j]; c.vry = vyi - a.v[n + j]; c.vrz = vzi - a.v[2 * n + j];
            c.wsx = ri * wxi + c.rb * a.w[j];
            c.wsy = ri * wyi + c.rb * a.w[n + j];
            c.wsz = ri * wzi + c.rb * a.w[2 * n + j];
            const PairCoef pc = coef[ti * s.ntypes + a.type[j]];
            double hx = 0.0, hy = 0.0, hz = 0.0;
            const int64_t slot = (int64_t)q * n + i;
            const int64_t plane = (int64_t)a.kmax * n;
            if ((mask >> q) & 1ull) {
                hx = L.xi[slot]; hy = L.xi[plane + slot]; hz = L.xi[2 * plane + slot];
            }
            double fx, fy, fz, tx, ty, tz, nx, ny, nz, fn;
            if (!contact_force(c, false, pc, s.dt, update != 0, hx, hy, hz, fx, fy, fz, tx, ty, tz, nx, ny, nz, fn))
                continue;
            if (COUNT) ++ncont;
            Fx = Fx + fx; Fy = Fy + fy; Fz = Fz + fz;
            Tx = Tx - ri * (ny * tz - nz * ty);
            Ty = Ty - ri * (nz * tx - nx * tz);
            Tz = Tz - ri * (nx * ty - ny * tx);
            if (update) {
                L.xi[slot] = hx; L.xi[plane + slot] = hy; L.xi[2 * plane + slot] = hz;
                nmask |= 1ull << q;
            }
        }
        if (s.wall && zi < ri) {
            ContactIn c;
            c.dx = 0.0; c.dy = 0.0; c.dz = zi;
            c.ra = ri; c.rb = 0.0; c.ma = mi; c.mb = 0.0;
            c.vrx = vxi; c.vry = vyi; c.vrz = vzi;
            c.wsx = ri * wxi; c.wsy = ri * wyi; c.wsz = ri * wzi;
            const PairCoef pc = coef[ti * s.ntypes + ti];
            double hx = 0.0, hy = 0.0, hz = 0.0;
            if (mask & kWallBit) { hx = a.xiw[i]; hy = a.xiw[n + i]; hz = a.xiw[2 * n + i]; }
            double fx, fy, fz, tx, ty, tz, nx, ny, nz, fn;
            if (contact_force(c, true, pc, s.dt, update != 0, hx, hy, hz, fx, fy, fz, tx, ty, tz, nx, ny, nz, fn)) {
                if (COUNT) ++nwall;
                Fx = Fx + fx; Fy = Fy + fy; Fz = Fz + fz;
                Tx = Tx - ri * (ny * tz - nz * ty);
                Ty = Ty - ri * (nz * tx - nx * tz);
                Tz = Tz - ri * (nx * ty - ny * tx);
                if (update) {
                    a.xiw[i] = hx; a.xiw[n + i] = hy; a.xiw[2 * n + i] = hz;
                    nmask |= kWallBit;
                }
            }
        }
        a.f[i] = Fx; a.f[n + i] = Fy; a.f[2 * n + i] = Fz;
        a.t[i] = Tx; a.t[n + i] = Ty; a.t[2 * n + i] = Tz;
        if (update && nmask != mask) L.mask[i] = nmask;
    }
    if (COUNT) {
        // statistics only (contact-pair rate); the force sums above use no atomics
        __shared__ unsigned long long sc[2];
        if (threadIdx.x == 0) { sc[0] = 0; sc[1] = 0; }
        __syncthreads();
        if (ncont) atomicAdd(&sc[0], (unsigned long long)ncont);
        if (nwall) atomicAdd(&sc[1], (unsigned long long)nwall);
        __syncthreads();
        if (threadIdx.x == 0) {
            if (sc[0]) atomicAdd(&a.flags->contacts, sc[0]);
            if (sc[1]) atomicAdd(&a.flags->wall_contacts, sc[1]);
        }
    }
}

// ------------------------------------------------------------------ binning

template <bool BATCH>
__global__ void k_bin_count(KArgs a) {
    const int64_t n = a.n;
    FOR_EACH_PARTICLE(n, i) {
        const SysDesc &s = a.sys[sys_of<BATCH>(a, i)];
        int cx = cell_coord(a.x[i], s, 0);
        int cy = cell_coord(a.x[n + i], s, 1);
        int cz = cell_coord(a.x[2 * n + i], s, 2);
        int64_t c = s.c0 + ((int64_t)cz * s.nc[1] + cy) * s.nc[0] + cx;
        a.cell_of[i] = (int32_t)c;
        a.rank[i] = atomicAdd(&a.cell_count[c], 1);
    }
}

// Exclusive scan of cell_count[0..m) into cell_start[0..m], three passes of
// 1024 elements per block.
constexpr int kScanBlock = 256, kScanItems = 4, kScanTile = kScanBlock * kScanItems;

__device__ inline int block_exclusive_scan(int v, int *lds, int &total) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int add = t >= off ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    total = lds[kScanBlock - 1];
    int ex = lds[t] - v;
    __syncthreads();
    return ex;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_partial(const int32_t *in, int64_t m, int32_t *partial) {
    __shared__ int lds[kScanBlock];
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < m) s += in[base + k];
    int total;
    block_exclusive_scan(s, lds, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_top(int32_t *partial, int64_t nb) {
    __shared__ int lds[kScanBlock];
    int carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        int64_t i = base + threadIdx.x;
        int v = i < nb ? partial[i] : 0;
        int total;
        int ex = block_exclusive_scan(v, lds, total);
        if (i < nb) partial[i] = carry + ex;
        carry += total;
    }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const int32_t *in, int64_t m, const int32_t *partial,
                                                           int32_t *out) {
    __shared__ int lds[kScanBlock];
    int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int vals[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = base + k < m ? in[base + k] : 0;
        s += vals[k];
    }
    int total;
    int ex = block_exclusive_scan(s, lds, total) + partial[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) out[base + k] = ex;
        ex += vals[k];
        if (base + k == m - 1) out[m] = ex;
    }
}

template <bool BATCH>
__global__ void k_bin_place(KArgs a) {
    FOR_EACH_PARTICLE(a.n, i) {
        int32_t c = a.cell_of[i];
        a.order[a.cell_start[c] + a.rank[i]] = (int32_t)i;
    }
}

// Order each cell's particles by id (insertion sort; cells are small).
__global__ void k_cell_sort(KArgs a) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < a.ncell;
         c += (int64_t)gridDim.x * blockDim.x) {
        int32_t b = a.cell_start[c], e = a.cell_start[c + 1];
        if (e - b > kCellSortMax) {
            atomicOr(&a.flags->err, kErrCellOverflow);
            continue;
        }
        for (int32_t p = b + 1; p < e; ++p) {
            int32_t v = a.order[p];
            int32_t idv = a.id[v];
            int32_t q = p - 1;
            while (q >= b && a.id[a.order[q]] > idv) {
                a.order[q + 1] = a.order[q];
                --q;
            }
            a.order[q + 1] = v;
        }
    }
}

// Gather every per-particle array into the shadow copy in the new order.
__global__ void k_gather(KArgs a, int frame_identity) {
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t src = a.order[i];
        double *sd = a.shadow_d;
        for (int c = 0; c < 3; ++c) {
            sd[(0 + c) * n + i] = a.x[c * n + src];
            sd[(3 + c) * n + i] = a.v[c * n + src];
            sd[(6 + c) * n + i] = a.w[c * n + src];
            sd[(9 + c) * n + i] = a.f[c * n + src];
            sd[(12 + c) * n + i] = a.t[c * n + src];
            sd[(15 + c) * n + i] = a.disp[c * n + src];
            sd[(18 + c) * n + i] = a.xiw[c * n + src];
        }
        sd[21 * n + i] = a.r[src];
        sd[22 * n + i] = a.m[src];
        sd[23 * n + i] = a.inv_m[src];
        sd[24 * n + i] = a.inv_I[src];
        int32_t *si = a.shadow_i;
        si[i] = a.type[src];
        si[n + i] = a.id[src];
        si[2 * n + i] = frame_identity ? (int32_t)src : a.frame[src];
    }
}

__global__ void k_scatter_back(KArgs a) {
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double *sd = a.shadow_d;
        for (int c = 0; c < 3; ++c) {
            a.x[c * n + i] = sd[(0 + c) * n + i];
            a.v[c * n + i] = sd[(3 + c) * n + i];
            a.w[c * n + i] = sd[(6 + c) * n + i];
            a.f[c * n + i] = sd[(9 + c) * n + i];
            a.t[c * n + i] = sd[(12 + c) * n + i];
            a.disp[c * n + i] = sd[(15 + c) * n + i];
            a.xiw[c * n + i] = sd[(18 + c) * n + i];
        }
        a.r[i] = sd[21 * n + i];
        a.m[i] = sd[22 * n + i];
        a.inv_m[i] = sd[23 * n + i];
        a.inv_I[i] = sd[24 * n + i];
        const int32_t *si = a.shadow_i;
        a.type[i] = si[i];
        a.id[i] = si[n + i];
        a.frame[i] = si[2 * n + i];
    }
}

// ------------------------------------------------------------ neighbour list

// Row of particle i: all j != i with d^2 < (r_i + r_j + skin)^2 in the 27
// surrounding cells, kept sorted by id in LDS while it is collected.  The
// history of pairs that were in the previous list is carried over by merging
// the two id-sorted rows.
template <bool BATCH>
__global__ void __launch_bounds__(256) k_neighbors(KArgs a, int have_old) {
    extern __shared__ int32_t lds[];
    const int64_t n = a.n;
    const int kmax = a.kmax;
    int32_t *rid = lds + threadIdx.x * 2 * kmax;
    int32_t *ridx = rid + kmax;
    int maxrow = 0;
    const List L = a.cur, O = a.old;
    const int64_t plane = (int64_t)kmax * n;
    FOR_EACH_PARTICLE(n, i) {
        const SysDesc &s = a.sys[sys_of<BATCH>(a, i)];
        const double xi = a.x[i], yi = a.x[n + i], zi = a.x[2 * n + i], ri = a.r[i];
        const int ccx = cell_coord(xi, s, 0), ccy = cell_coord(yi, s, 1), ccz = cell_coord(zi, s, 2);
        int count = 0;
        for (int dz = -1; dz <= 1; ++dz) {
            int cz = ccz + dz;
            if (s.periodic[2]) { cz = cz < 0 ? cz + s.nc[2] : (cz >= s.nc[2] ? cz - s.nc[2] : cz); if (s.nc[2] < 3 && dz == -1) continue; }
            else if (cz < 0 || cz >= s.nc[2]) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                int cy = ccy + dy;
                if (s.periodic[1]) { cy = cy < 0 ? cy + s.nc[1] : (cy >= s.nc[1] ? cy - s.nc[1] : cy); if (s.nc[1] < 3 && dy == -1) continue; }
                else if (cy < 0 || cy >= s.nc[1]) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    int cx = ccx + dx;
                    if (s.periodic[0]) { cx = cx < 0 ? cx + s.nc[0] : (cx >= s.nc[0] ? cx - s.nc[0] : cx); if (s.nc[0] < 3 && dx == -1) continue; }
                    else if (cx < 0 || cx >= s.nc[0]) continue;
                    const int64_t c = s.c0 + ((int64_t)cz * s.nc[1] + cy) * s.nc[0] + cx;
                    const int32_t b = a.cell_start[c], e = a.cell_start[c + 1];
                    for (int32_t j = b; j < e; ++j) {
                        if (j == i) continue;
                        double ddx = min_image(xi - a.x[j], s.L[0], s.hL[0], s.periodic[0]);
                        double ddy = min_image(yi - a.x[n + j], s.L[1], s.hL[1], s.periodic[1]);
                        double ddz = min_image(zi - a.x[2 * n + j], s.L[2], s.hL[2], s.periodic[2]);
                        double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        double cut = ri + a.r[j] + s.skin;
                        if (!(d2 < cut * cut)) continue;
                        if (count < kmax) {
                            int32_t idj = a.id[j];
                            int q = count - 1;
                            while (q >= 0 && rid[q] > idj) {
                                rid[q + 1] = rid[q];
                                ridx[q + 1] = ridx[q];
                                --q;
                            }
                            rid[q + 1] = idj;
                            ridx[q + 1] = j;
                        }
                        ++count;
                    }
                }
            }
        }
        if (count > maxrow) maxrow = count;
        const int cnt = count < kmax ? count : kmax;
        uint64_t nmask = 0;
        if (have_old) {
            const int64_t o = a.frame[i];
            const int ocnt = O.cnt[o];
            const uint64_t omask = O.mask[o];
            nmask = omask & kWallBit;
            int p = 0;
            for (int q = 0; q < cnt; ++q) {
                const int32_t idq = rid[q];
                while (p < ocnt && O.ids[O.nbr[(int64_t)p * n + o]] < idq) ++p;
                if (p < ocnt && O.ids[O.nbr[(int64_t)p * n + o]] == idq && ((omask >> p) & 1ull)) {
                    const int64_t os = (int64_t)p * n + o, ns = (int64_t)q * n + i;
                    L.xi[ns] = O.xi[os];
                    L.xi[plane + ns] = O.xi[plane + os];
                    L.xi[2 * plane + ns] = O.xi[2 * plane + os];
                    nmask |= 1ull << q;
                }
            }
        }
        for (int q = 0; q < cnt; ++q) L.nbr[(int64_t)q * n + i] = ridx[q];
        L.cnt[i] = cnt;
        L.mask[i] = nmask;
        L.ids[i] = a.id[i];
        a.disp[i] = 0.0; a.disp[n + i] = 0.0; a.disp[2 * n + i] = 0.0;
    }
    if (maxrow > kmax) atomicOr(&a.flags->err, kErrCapacity);
    if (maxrow) atomicMax(&a.flags->max_row, maxrow);
}

// ------------------------------------------------------------------ launchers

static int grid_for(int64_t n, int block) {
    int64_t tiles = (n + block - 1) / block;
    int64_t g = (tiles + kXcd - 1) / kXcd * kXcd;
    const int64_t cap = 256 * kXcd;  // persistent: at most 8 waves of tiles per XCD slot
    if (g > cap) g = cap;
    if (g < kXcd) g = kXcd;
    return (int)g;
}

static int flat_grid(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

#define CHECK_LAUNCH() return hipGetLastError()

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<flat_grid(n, 256), 256, 0, st>>>(p, n, v);
    CHECK_LAUNCH();
}
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill_u64<<<flat_grid(n, 256), 256, 0, st>>>(p, n, v);
    CHECK_LAUNCH();
}
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill_f64<<<flat_grid(n, 256), 256, 0, st>>>(p, n, v);
    CHECK_LAUNCH();
}
hipError_t launch_ctrl(Flags *f, int op, int64_t value, hipStream_t st) {
    k_ctrl<<<1, 64, 0, st>>>(f, op, value);
    CHECK_LAUNCH();
}

hipError_t launch_init_mass(const KArgs &a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    if (a.nsys > 1) k_init_mass<true><<<grid_for(a.n, a.block), a.block, 0, st>>>(a);
    else k_init_mass<false><<<grid_for(a.n, a.block), a.block, 0, st>>>(a);
    CHECK_LAUNCH();
}

hipError_t launch_phase(const KArgs &a, int phase, int k, int gate, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    const int g = grid_for(a.n, a.block);
    if (phase == 0) {
        if (a.nsys > 1) k_phase0<true><<<g, a.block, 0, st>>>(a, k, gate);
        else k_phase0<false><<<g, a.block, 0, st>>>(a, k, gate);
    } else {
        if (a.nsys > 1) k_phase1<true><<<g, a.block, 0, st>>>(a, k, gate);
        else k_phase1<false><<<g, a.block, 0, st>>>(a, k, gate);
    }
    CHECK_LAUNCH();
}

hipError_t launch_forces(const KArgs &a, int update, int k, int gate, int count, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    const int g = grid_for(a.n, a.block);
    if (a.nsys > 1) {
        if (count) k_forces<true, true><<<g, a.block, 0, st>>>(a, update, k, gate);
        else k_forces<true, false><<<g, a.block, 0, st>>>(a, update, k, gate);
    } else {
        if (count) k_forces<false, true><<<g, a.block, 0, st>>>(a, update, k, gate);
        else k_forces<false, false><<<g, a.block, 0, st>>>(a, update, k, gate);
    }
    CHECK_LAUNCH();
}

hipError_t launch_bin(const KArgs &a, int frame_identity, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipError_t e;
    if ((e = launch_fill_i32(a.cell_count, a.ncell + 1, 0, st)) != hipSuccess) return e;
    const int g = grid_for(a.n, a.block);
    if (a.nsys > 1) k_bin_count<true><<<g, a.block, 0, st>>>(a);
    else k_bin_count<false><<<g, a.block, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t m = a.ncell;
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    k_scan_partial<<<(int)nb, kScanBlock, 0, st>>>(a.cell_count, m, a.scan_partial);
    k_scan_top<<<1, kScanBlock, 0, st>>>(a.scan_partial, nb);
    k_scan_apply<<<(int)nb, kScanBlock, 0, st>>>(a.cell_count, m, a.scan_partial, a.cell_start);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.nsys > 1) k_bin_place<true><<<g, a.block, 0, st>>>(a);
    else k_bin_place<false><<<g, a.block, 0, st>>>(a);
    k_cell_sort<<<flat_grid(m, 256), 256, 0, st>>>(a);
    k_gather<<<flat_grid(a.n, 256), 256, 0, st>>>(a, frame_identity);
    k_scatter_back<<<flat_grid(a.n, 256), 256, 0, st>>>(a);
    CHECK_LAUNCH();
}

hipError_t launch_neighbors(const KArgs &a, int have_old, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    // two LDS rows of kmax ints per thread; keep the workgroup at <= 32 KB
    const int block = a.kmax > 32 ? 64 : 128;
    const size_t lds = (size_t)block * 2 * a.kmax * sizeof(int32_t);
    const int g = grid_for(a.n, block);
    if (a.nsys > 1) k_neighbors<true><<<g, block, lds, st>>>(a, have_old);
    else k_neighbors<false><<<g, block, lds, st>>>(a, have_old);
    CHECK_LAUNCH();
}

}  // namespace dem
