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

// The same over the particle window [a.w0, a.w1) of the rebuild kernels.
#define FOR_EACH_IN_WINDOW(a, i)                                                        \
    for (TileIter _it = tiles((a).w1 - (a).w0); _it.t < _it.tend; _it.t += _it.stride) \
        for (int64_t i = (a).w0 + _it.t * blockDim.x + threadIdx.x; i < (a).w1; i = (a).w1)

#define FOR_WINDOW_FLAT(a, i)                                                                       \
    for (int64_t i = (a).w0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (a).w1;            \
         i += (int64_t)gridDim.x * blockDim.x)

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

__device__ inline int sys_of_any(const KArgs &a, int64_t i) {
    int lo = 0, hi = a.nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (i < a.sys[mid].p1) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ inline List list_of(const KArgs &a, int sy, int which) {
    // which 0: the system's current list, 1: its other buffer
    const int b = a.lcur[sy] ^ which;
    return b ? a.lst[1] : a.lst[0];
}

__device__ inline int sys_of_cell(const KArgs &a, int64_t c) {
    int lo = 0, hi = a.nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.sys[mid].c0 <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
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
// op 4: builds += value; op 5: call_base = value; op 6: step_end = value
__global__ void k_ctrl(Flags *f, int op, int64_t value) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    if (op == 0) { f->abort_at = INT64_MAX; f->step_base = value; }
    else if (op == 1) { f->step_base += value; }
    else if (op == 2) {
        f->err = 0; f->max_row = 0; f->abort_at = INT64_MAX; f->step_base = 0;
        f->steps = 0; f->builds = 0; f->contacts = 0; f->wall_contacts = 0;
    } else if (op == 3) { f->steps += value; }
    else if (op == 4) { f->builds += value; }
    else if (op == 5) { f->call_base = value; }
    else if (op == 6) { f->step_end = value; }
}

// Multi-rate stepping: the packed buffer that holds a system's state at
// substep qa (1-based) of a call, i.e. after the drift into its next step:
// the parity of the number of its steps before qa.
__device__ inline int mr_buffer(int64_t qa, int stride) {
    return (int)(((qa - 1 + stride - 1) / stride) & 1);
}

// ------------------------------------------------------------------ masses

// Also validates what later kernels index with: type in [0, ntypes), id >= 0,
// r > 0 (a bad particle is flagged and its type forced to 0).
template <bool BATCH>
__global__ void k_init_mass(KArgs a) {
    bool bad = false;
    FOR_EACH_PARTICLE(a.n, i) {
        const SysDesc &s = a.sys[sys_of<BATCH>(a, i)];
        if (i >= s.pe) continue;   // a free slot
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
        if (i >= s.pe) continue;
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
        if (i >= s.pe) continue;
        double im = a.inv_m[i], iI = a.inv_I[i];
        for (int c = 0; c < 3; ++c) {
            a.v[c * n + i] = a.v[c * n + i] + s.hdt * (a.f[c * n + i] * im);
            a.w[c * n + i] = a.w[c * n + i] + s.hdt * (a.t[c * n + i] * iI);
        }
    }
}

// ------------------------------------------------------------------ binning

// Counts of the selected systems' cells only: the other systems keep the
// counts of their own last binning, so that cell_start (one scan over all
// cells) still gives every system the particle range of each of its cells in
// the order it keeps until its next rebuild.
// A system's spare cell starts with its free slots (placed without atomics,
// in slot order); removed particles are counted in after them.
__global__ void k_zero_selected_cells(KArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cell_count[a.ncell] = 0;
    for (int64_t c = a.cw0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < a.cw1;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int sy = sys_of_cell(a, c);
        if (!a.sel[sy]) continue;
        const SysDesc &s = a.sys[sy];
        const bool spare = c == s.c0 + (int64_t)s.nc[0] * s.nc[1] * s.nc[2];
        a.cell_count[c] = spare ? (int32_t)(s.p1 - s.pe) : 0;
    }
}

template <bool BATCH>
__global__ void k_bin_count(KArgs a) {
    const int64_t n = a.n;
    FOR_EACH_IN_WINDOW(a, i) {
        const int sy = sys_of<BATCH>(a, i);
        if (!a.sel[sy]) continue;
        const SysDesc &s = a.sys[sy];
        // free slots and removed particles go to the spare cell past the grid:
        // the free slots first, in slot order (no atomics: a system may hold
        // many), then the removed ones (removal marks are consumed here)
        const int64_t spare = s.c0 + (int64_t)s.nc[0] * s.nc[1] * s.nc[2];
        if (i >= s.pe) {
            a.cell_of[i] = (int32_t)spare;
            a.rank[i] = (int32_t)(i - s.pe);
            continue;
        }
        int64_t c = spare;
        if (a.dead[i]) {
            a.dead[i] = 0;
        } else {
            int cx = cell_coord(a.x[i], s, 0);
            int cy = cell_coord(a.x[n + i], s, 1);
            int cz = cell_coord(a.x[2 * n + i], s, 2);
            c = s.c0 + ((int64_t)cz * s.nc[1] + cy) * s.nc[0] + cx;
        }
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

// Particles of the systems selected for a rebuild go to their cell's range;
// the others keep their place (their list is kept, not rebuilt).
template <bool BATCH>
__global__ void k_bin_place(KArgs a) {
    FOR_EACH_IN_WINDOW(a, i) {
        if (!a.sel[sys_of<BATCH>(a, i)]) continue;
        int32_t c = a.cell_of[i];
        a.order[a.cell_start[c] + a.rank[i]] = (int32_t)i;
    }
}

// Order each cell's particles by id (insertion sort; cells are small).
__global__ void k_cell_sort(KArgs a) {
    for (int64_t c = a.cw0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < a.cw1;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int sy = sys_of_cell(a, c);
        if (!a.sel[sy]) continue;
        const SysDesc &s = a.sys[sy];
        if (c == s.c0 + (int64_t)s.nc[0] * s.nc[1] * s.nc[2]) continue;   // the spare cell: free slots
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
    FOR_WINDOW_FLAT(a, i) {
        if (!a.sel[sys_of_any(a, i)]) continue;  // not rebuilt: stays in place
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
        if (a.fext)
            for (int c = 0; c < 3; ++c) sd[(25 + c) * n + i] = a.fext_ws[c * n + src];
        int32_t *si = a.shadow_i;
        si[i] = a.type[src];
        si[n + i] = a.id[src];
        si[2 * n + i] = frame_identity ? (int32_t)src : a.frame[src];
        if (a.sxi) {
            double *ss = a.shadow_s;
            for (int k = 0; k < a.nsurf_slots; ++k) {
                const D4 h = a.sxi[k * n + src];
                ss[(3 * k) * n + i] = h.x;
                ss[(3 * k + 1) * n + i] = h.y;
                ss[(3 * k + 2) * n + i] = h.z;
            }
            ((uint32_t *)(ss + 3 * a.nsurf_slots * n))[i] = a.smask[src];
        }
    }
}

__global__ void k_scatter_back(KArgs a) {
    const int64_t n = a.n;
    FOR_WINDOW_FLAT(a, i) {
        if (!a.sel[sys_of_any(a, i)]) continue;
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
        if (a.fext)
            for (int c = 0; c < 3; ++c) a.fext_ws[c * n + i] = sd[(25 + c) * n + i];
        const int32_t *si = a.shadow_i;
        a.type[i] = si[i];
        a.id[i] = si[n + i];
        a.frame[i] = si[2 * n + i];
        if (a.sxi) {
            const double *ss = a.shadow_s;
            for (int k = 0; k < a.nsurf_slots; ++k)
                a.sxi[k * n + i] = D4{ss[(3 * k) * n + i], ss[(3 * k + 1) * n + i], ss[(3 * k + 2) * n + i], 0.0};
            a.smask[i] = ((const uint32_t *)(ss + 3 * a.nsurf_slots * n))[i];
        }
    }
}

// ------------------------------------------------------------ neighbour list

// Row of particle i: all j != i with d^2 < (r_i + r_j + skin)^2 in the 27
// surrounding cells, sorted by id.  A group of kNbrLanes lanes per particle.
// The three cells along x of each (dz, dy) row of cells are one run of
// candidates (two pieces where the run crosses a periodic seam in x).  Each
// lane reads the bounds of three of the nine runs into the group's LDS table,
// with no branch between the loads, so that they are in flight together.
// Each group deals its candidates to its lanes in turn, kNbrUnroll per lane
// loaded before any is tested; hits are appended to the group's LDS buffer in
// candidate order (a ballot gives each its place).
// Then the hits' ids are fetched, each lane ranks its entries by id (ids are
// unique) and writes them to their places in the row, and the history of
// pairs of the previous list is carried over by id (binary search of the
// previous row, also sorted by id).  A group's LDS buffers are its own and
// its lanes share a wave, so no barrier spans the block until the end.
//
// Measured on the 1e6-sphere bed (ms per build), with the run bounds held in
// registers (117 of them, four waves per SIMD): 4 lanes per particle 0.48,
// against 0.51 for 2, 0.61 for 8, 0.80 for 1 and 0.90 for 16; two candidates
// per lane in flight against one 0.52 and four (which spill) 0.52.  With the
// run table in LDS the kernel needs 95 registers and runs five waves per
// SIMD: 0.41 (six waves spill: 0.42).
constexpr int kNbrLanes = 4;
constexpr int kNbrBlock = 256;
static_assert(3 * kNbrLanes >= 9, "each lane reads the bounds of at most three of the nine runs");
constexpr int kNbrUnroll = 2;

// LDS of k_neighbors, per group: its hits' indices (kmax words), then their
// ids and the previous row's ids (kmax each), over which the table of the nine
// runs (3 words each) lies during the collection; an odd number of words, so
// that the groups of a wave start in different banks.
__host__ __device__ inline int nbr_group_words(int kmax) {
    const int w = kmax + (2 * kmax > 27 ? 2 * kmax : 27);
    return w | 1;
}
__host__ __device__ inline size_t nbr_lds_bytes(int kmax, int block) {
    return (size_t)nbr_group_words(kmax) * (block / kNbrLanes) * sizeof(int32_t);
}

// Orders the LDS accesses of one wave's lanes (the buffers a group shares).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entry q of a group's hits: its rank by id gives its slot in the new row,
// where its index is written; returns whether the previous row (ids oid,
// sorted) holds the pair with a history, and then where (from).
__device__ __forceinline__ bool nbr_place(const int32_t *bid, const int32_t *bidx, const int32_t *oid, int cnt,
                                          int ocnt, uint64_t omask, int have_old, int64_t n, int64_t i, int64_t o,
                                          int kmax, const List &L, int q, int64_t &slot, int64_t &from,
                                          uint64_t &bits) {
    const int32_t idq = bid[q];
    int rank = 0;
    for (int k = 0; k < cnt; ++k) rank += bid[k] < idq ? 1 : 0;
    slot = i * kmax + rank;
    L.nbr[rank * n + i] = bidx[q];
    if (!have_old) return false;
    int lo = 0, hi = ocnt;   // first p with oid[p] >= idq
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (oid[mid] < idq) lo = mid + 1;
        else hi = mid;
    }
    if (lo < ocnt && oid[lo] == idq && ((omask >> lo) & 1ull)) {
        from = o * kmax + lo;
        bits |= 1ull << rank;
        return true;
    }
    return false;
}

template <bool BATCH>
__global__ void __launch_bounds__(kNbrBlock, 5) k_neighbors(KArgs a, int have_old) {
    extern __shared__ int32_t nbr_lds[];
    __shared__ int32_t blockmax;
    constexpr int G = kNbrLanes;
    const int64_t n = a.n;
    const int kmax = a.kmax;
    const int g = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int ppb = blockDim.x / G;
    const int gbase = (threadIdx.x % warpSize) / G * G;
    const uint64_t gmask = (1ull << G) - 1;
    int32_t *bidx = nbr_lds + grp * nbr_group_words(kmax);   // the group's hits' indices
    int32_t *bid = bidx + kmax;                               //   their ids
    int32_t *oid = bid + kmax;                                //   the previous row's ids
    int32_t *runs = bid;                                      //   the nine runs, while collecting
    const D4 *Q = (const D4 *)a.shadow_d;  // (x, y, z, r) in the current order (k_nbr_pack)
    const int32_t *cs = a.cell_start;
    const int64_t ntiles = (a.w1 - a.w0 + ppb - 1) / ppb;
    const int per = gridDim.x / kXcd;
    const int64_t chunk = (ntiles + kXcd - 1) / kXcd;
    const int64_t t0 = (blockIdx.x % kXcd) * chunk;
    const int64_t t1 = t0 + chunk < ntiles ? t0 + chunk : ntiles;
    int maxrow = 0;
    for (int64_t t = t0 + blockIdx.x / kXcd; t < t1; t += per) {
        const int64_t i = a.w0 + t * ppb + grp;
        int sy = 0;
        bool active = i < a.w1;
        // the particle's own record and its previous position, loaded before the
        // selection test so that the loads overlap
        const int64_t ic = active ? i : 0;
        const D4 qi = Q[ic];
        const int64_t o0 = have_old ? a.frame[ic] : 0;
        if (active) {
            sy = sys_of<BATCH>(a, i);
            // else the system keeps its list, or the slot is free
            active = a.sel[sy] != 0 && i < a.sys[sy].pe;
        }
        // a particle inserted since the last build has no previous row
        const int old_i = have_old && o0 >= 0;
        const int64_t o = old_i ? o0 : 0;
        int count = 0;
        if (active) {
            const SysDesc &s = a.sys[sy];
            const int nx = s.nc[0], ny = s.nc[1], nz = s.nc[2];
            const int px = s.periodic[0], py = s.periodic[1], pz = s.periodic[2];
            const int ccx = cell_coord(qi.x, s, 0), ccy = cell_coord(qi.y, s, 1), ccz = cell_coord(qi.z, s, 2);
            // Within one row of cells that does not wrap, |d| < 2 cell widths; on an
            // axis of five or more cells that is under half the box, where the
            // minimum image is d itself, so it is only taken where a row can wrap.
            const bool mix = px && (nx < 5 || ccx == 0 || ccx == nx - 1);
            // cells x0 .. x1 of each row, and on a periodic axis of three or more
            // cells at its seam, the cell c2 across it (else c2 = x0, no second piece)
            const bool wrapx = px && nx >= 3;
            const bool seam = wrapx && (ccx == 0 || ccx == nx - 1);
            const int x0 = wrapx ? (ccx == 0 ? 0 : ccx - 1) : (ccx > 0 ? ccx - 1 : 0);
            const int x1 = wrapx ? (ccx == nx - 1 ? nx - 1 : ccx + 1) : (ccx + 1 < nx ? ccx + 1 : nx - 1);
            const int c2 = seam ? (ccx == 0 ? nx - 1 : 0) : x0;
            // minimum-image flags of the nine runs (every lane), then the runs'
            // bounds, each lane reading those of runs g, g + G, g + 2 G into the
            // group's LDS table (first index of each piece, length of the first)
            uint32_t my = 0, mz = 0;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int dz = k / 3 - 1, dy = k % 3 - 1;
                const int cz = ccz + dz, cy = ccy + dy;
                if (pz && (nz < 5 || cz < 0 || cz >= nz)) mz |= 1u << k;
                if (py && (ny < 5 || cy < 0 || cy >= ny)) my |= 1u << k;
            }
            int32_t lt[3] = {0, 0, 0};   // whole length of this lane's runs g, g + G, g + 2 G
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int k = g + r * G;
                if (k >= 9) break;
                const int dz = k / 3 - 1, dy = k % 3 - 1;
                int cz = ccz + dz, cy = ccy + dy;
                bool ok = true;
                if (pz) {
                    cz = cz < 0 ? cz + nz : (cz >= nz ? cz - nz : cz);
                    if (nz < 3 && dz == -1) ok = false;
                } else if (cz < 0 || cz >= nz) ok = false;
                if (py) {
                    cy = cy < 0 ? cy + ny : (cy >= ny ? cy - ny : cy);
                    if (ny < 3 && dy == -1) ok = false;
                } else if (cy < 0 || cy >= ny) ok = false;
                const int64_t crow = s.c0 + (ok ? ((int64_t)cz * ny + cy) * nx : 0);   // a valid row either way
                const int32_t b1 = cs[crow + x0], e1 = cs[crow + x1 + 1];
                const int32_t b2 = cs[crow + c2], e2 = cs[crow + c2 + 1];
                const int32_t l1 = ok ? e1 - b1 : 0, l2 = ok && seam ? e2 - b2 : 0;
                runs[3 * k] = b1;
                runs[3 * k + 1] = b2;
                runs[3 * k + 2] = l1;
                lt[r] = l1 + l2;
            }
            wave_sync();
            // the runs' lengths from the lanes that read them, and their prefix
            int32_t pre[10];
            int total = 0;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                pre[k] = total;
                total += __shfl(lt[k / G], gbase + k % G);
            }
            pre[9] = total;
            // the system's constants in registers: the loop stores to LDS, and the
            // compiler would otherwise read them again from the table every round
            const double Lx = s.L[0], Ly = s.L[1], Lz = s.L[2];
            const double hx = s.hL[0], hy = s.hL[1], hz = s.hL[2], skin = s.skin;
            for (int v0 = 0; v0 < total; v0 += G * kNbrUnroll) {   // same trip count for the group
                D4 qj[kNbrUnroll];
                int32_t jj[kNbrUnroll], kk[kNbrUnroll];
#pragma unroll
                for (int e = 0; e < kNbrUnroll; ++e) {
                    const int v = v0 + e * G + g;
                    int32_t p0k = 0, k = 0;
#pragma unroll
                    for (int m = 1; m < 9; ++m)
                        if (v >= pre[m]) { p0k = pre[m]; k = m; }
                    const int32_t b1 = runs[3 * k], b2 = runs[3 * k + 1], l1 = runs[3 * k + 2];
                    const int u = v - p0k;
                    // past the end: the particle itself, which is no hit
                    jj[e] = v < total ? (u < l1 ? b1 + u : b2 + (u - l1)) : (int32_t)i;
                    kk[e] = k;
                    qj[e] = Q[jj[e]];
                }
#pragma unroll
                for (int e = 0; e < kNbrUnroll; ++e) {
                    const int32_t j = jj[e];
                    bool hit = false;
                    if (j != i) {
                        double ddx = qi.x - qj[e].x, ddy = qi.y - qj[e].y, ddz = qi.z - qj[e].z;
                        if (mix) ddx = min_image(ddx, Lx, hx, px);
                        if ((my >> kk[e]) & 1u) ddy = min_image(ddy, Ly, hy, py);
                        if ((mz >> kk[e]) & 1u) ddz = min_image(ddz, Lz, hz, pz);
                        const double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        const double cut = qi.w + qj[e].w + skin;
                        hit = d2 < cut * cut;
                    }
                    const uint64_t bal = (__ballot(hit) >> gbase) & gmask;
                    if (hit) {
                        const int pos = count + __popcll(bal & ((1ull << g) - 1));
                        if (pos < kmax) bidx[pos] = j;
                    }
                    count += __popcll(bal);
                }
            }
        }
        wave_sync();
        // ---- the hits' ids and the previous row's ids, all loads in flight at once
        const int cnt = count < kmax ? count : kmax;
        int ocnt = 0;
        uint64_t omask = 0;
        // (each lane takes two entries per round, both loads issued before either
        // is used: a row of up to 2 G entries is one round trip)
        if (active) {
            for (int q0 = g; q0 < cnt; q0 += 2 * G) {
                const int q1 = q0 + G;
                const int32_t j0 = bidx[q0], j1 = q1 < cnt ? bidx[q1] : j0;
                const int32_t id0 = a.id[j0], id1 = a.id[j1];
                bid[q0] = id0;
                if (q1 < cnt) bid[q1] = id1;
            }
            if (old_i) {
                const List O = list_of(a, sy, 0);
                ocnt = O.cnt[o];
                omask = O.mask[o];
                const int32_t *orow = O.nbr + o;   // entry p at orow[p n]
                for (int p0 = g; p0 < ocnt; p0 += 2 * G) {
                    const int p1 = p0 + G;
                    const int32_t j0 = orow[p0 * n], j1 = orow[(p1 < ocnt ? p1 : p0) * n];
                    const int32_t id0 = O.ids[j0], id1 = O.ids[j1];
                    oid[p0] = id0;
                    if (p1 < ocnt) oid[p1] = id1;
                }
            }
        }
        wave_sync();
        // ---- ranks, the row, and the history carried over
        if (active) {
            const List O = list_of(a, sy, 0), L = list_of(a, sy, 1);
            uint64_t bits = 0;
            for (int q0 = g; q0 < cnt; q0 += 2 * G) {
                const int q1 = q0 + G;
                int64_t s0, s1 = 0, f0, f1 = 0;
                const bool c0 = nbr_place(bid, bidx, oid, cnt, ocnt, omask, old_i, n, i, o, kmax, L, q0, s0, f0,
                                          bits);
                const bool c1 = q1 < cnt && nbr_place(bid, bidx, oid, cnt, ocnt, omask, old_i, n, i, o, kmax, L, q1,
                                                      s1, f1, bits);
                // both loads unconditional (slot 0 where nothing is carried), so that
                // they are issued together
                const D4 *p0 = O.xi + (c0 ? f0 : 0), *p1 = O.xi + (c1 ? f1 : 0);
                const double x0 = p0->x, y0 = p0->y, z0 = p0->z, w0 = p0->w;
                const double x1 = p1->x, y1 = p1->y, z1 = p1->z, w1 = p1->w;
                if (c0) L.xi[s0] = D4{x0, y0, z0, w0};
                if (c1) L.xi[s1] = D4{x1, y1, z1, w1};
            }
            for (int off = 1; off < G; off <<= 1) bits |= __shfl_xor(bits, off);
            if (g == 0) {
                if (count > maxrow) maxrow = count;
                L.cnt[i] = cnt;
                L.mask[i] = bits | (omask & kWallBit);
                L.ids[i] = a.id[i];
                a.disp[i] = 0.0; a.disp[n + i] = 0.0; a.disp[2 * n + i] = 0.0;
            }
        }
        wave_sync();   // the group's buffers are reused by the next tile
    }
    // the longest row: reduced over the block first, then one atomic per block
    // (one per particle, all on one address, serialised and cost about as much
    // as the whole build)
    if (threadIdx.x == 0) blockmax = 0;
    __syncthreads();
    if (maxrow) atomicMax(&blockmax, maxrow);
    __syncthreads();
    if (threadIdx.x == 0 && blockmax) {
        if (blockmax > kmax) atomicOr(&a.flags->err, kErrCapacity);
        atomicMax(&a.flags->max_row, blockmax);
    }
}

// After a build: the selected systems switch to the buffer just written.
__global__ void k_flip(KArgs a) {
    for (int sy = threadIdx.x; sy < a.nsys; sy += blockDim.x)
        if (a.sel[sy]) a.lcur[sy] ^= 1;
}

// ------------------------------------------------------------- fused step

// Caller arrays (structure of arrays) -> packed buffer `dst`.  mode 1 also
// does phase 0 of velocity Verlet for the step step_base + k (gated like the
// fused step: it asks for a rebuild when the displacement exceeds skin/2).
template <bool BATCH>
__global__ void k_pack(KArgs a, int dst, int mode, int k, int gate, int64_t qa) {
    int64_t step = 0;
    if (gate) {
        step = a.flags->step_base + k;
        if (a.flags->abort_at < step) return;
    }
    const int64_t n = a.n;
    bool need = false, bad = false;
    FOR_EACH_IN_WINDOW(a, i) {
        const int sy = sys_of<BATCH>(a, i);
        if (mode == 2 && !a.sel[sy]) continue;
        const SysDesc &s = a.sys[sy];
        if (i >= s.pe) continue;   // a free slot
        const int d = mode == 2 && a.multirate ? mr_buffer(qa, s.stride) : dst;
        D4 *P = a.pos[d], *V = a.vel[d], *S = a.spin[d];
        const double im = a.inv_m[i], iI = a.inv_I[i];
        double x[3], v[3], w[3];
        for (int c = 0; c < 3; ++c) {
            x[c] = a.x[c * n + i];
            v[c] = a.v[c * n + i];
            w[c] = a.w[c * n + i];
        }
        if (mode == 1) {
            double dsq = 0.0;
            for (int c = 0; c < 3; ++c) {
                v[c] = v[c] + s.hdt * (a.f[c * n + i] * im);
                w[c] = w[c] + s.hdt * (a.t[c * n + i] * iI);
                x[c] = wrap_axis(x[c] + s.dt * v[c], s, c);
                const double d = a.disp[c * n + i] + s.dt * v[c];
                a.disp[c * n + i] = d;
                dsq += d * d;
            }
            if (!(dsq <= s.disp_thr2)) {
                need = true;
                a.sel[sys_of<BATCH>(a, i)] = 1;
            }
            if (!isfinite(x[0] + x[1] + x[2] + v[0] + v[1] + v[2])) bad = true;
        }
        P[i] = D4{x[0], x[1], x[2], a.r[i]};
        V[i] = D4{v[0], v[1], v[2], a.m[i]};
        S[i] = D4{w[0], w[1], w[2], (double)(sy * 16 + a.type[i])};  // system and type in one exact code
        a.im[i] = D2{im, iI};
    }
    if (bad) atomicOr(&a.flags->err, kErrNonFinite);
    if (need && gate) a.flags->abort_at = step;
}

// Packed buffer `src` -> caller arrays x, v, w (with selected: only the
// systems selected for a rebuild).
__global__ void k_unpack(KArgs a, int src, int selected, int64_t qa) {
    const int64_t n = a.n;
    FOR_WINDOW_FLAT(a, i) {
        const int sy = sys_of_any(a, i);
        if (selected && !a.sel[sy]) continue;
        if (i >= a.sys[sy].pe) continue;
        const int b = a.multirate && qa > 0 ? mr_buffer(qa, a.sys[sy].stride) : src;
        const D4 p = a.pos[b][i], v = a.vel[b][i], w = a.spin[b][i];
        a.x[i] = p.x; a.x[n + i] = p.y; a.x[2 * n + i] = p.z;
        a.v[i] = v.x; a.v[n + i] = v.y; a.v[2 * n + i] = v.z;
        a.w[i] = w.x; a.w[n + i] = w.y; a.w[2 * n + i] = w.z;
    }
}

// Force pass over the packed state in buffer src, one group of G lanes per
// particle (lane g of the group takes slots g, g+G, ... of the row), so a
// whole row's loads are in flight at once.  The pair terms (contact_force,
// Eq. (3)-(6)) are computed in parallel and then added in ascending slot
// order -- the row is sorted by neighbour id -- by every lane of the group,
// reading each term from its lane: per particle the sum is gravity, then the
// contacts in ascending neighbour id, then the wall, exactly the sequential
// order, whatever the list composition, the lanes or the block size.
//   MODE 0: forces only, written to f and t (history advanced when update);
//   MODE 1: fused step -- forces, kick 1/2, then the next step's kick 1/2,
//           drift, wrap and rebuild check, written to buffer src^1 (gated:
//           does nothing once an earlier step asked for a rebuild);
//   MODE 2: last step of a call -- forces, kick 1/2, and f, t, x, v, w
//           written to the caller's arrays (gated).
// The block's system's pair coefficients (ntypes x ntypes): read by every
// contact, so kept in LDS instead of three global loads per contact.
__shared__ PairCoef step_coef[kMaxTypes * kMaxTypes];

__device__ __forceinline__ void load_step_coef(const KArgs &a, const SysDesc &s) {
    __syncthreads();   // readers of the previous table are done
    for (int k = threadIdx.x; k < s.ntypes * s.ntypes; k += blockDim.x) step_coef[k] = a.coef[s.coef0 + k];
    __syncthreads();
}

// One particle of the force pass (see k_step): every lane of its group calls
// this with the same i; s is the particle's system (the block's: a tile never
// spans two systems), L its current list.
template <bool BATCH, bool COUNT, int MODE, int G, bool MR, bool SURF>
__device__ __forceinline__ void step_particle(const KArgs &a, const SysDesc &s, const List &L, int src, int update,
                                              int64_t i, int sy, const D4 &pi, const D4 &vi, const D4 &si, int code,
                                              int g, int gbase, uint64_t gmask, unsigned &ncont, unsigned &nwall,
                                              bool &need, bool &bad, bool last) {
    const int64_t n = a.n;
    const D4 *__restrict__ P = a.pos[src];
    const D4 *__restrict__ V = a.vel[src];
    const D4 *__restrict__ S = a.spin[src];
    const int64_t kmax = a.kmax;
        const int ti = code & 15;
        const PairCoef *coef = step_coef;   // the system's table, in LDS
        const double ri = pi.w, mi = vi.w;
        double Fx = mi * s.g[0], Fy = mi * s.g[1], Fz = mi * s.g[2];
        double Tx = 0.0, Ty = 0.0, Tz = 0.0;
        const int cnt = L.cnt[i];
        const uint64_t mask = L.mask[i];
        uint64_t nmask = 0;
        // the neighbour index of the lane's next chunk is loaded one chunk ahead, so
        // that its latency overlaps the current contact (294 -> 288 us per step on
        // the 1e6-sphere bed; loading the velocity, spin and history before the
        // contact test as well spills and was slower)
        int32_t jn = g < cnt ? L.nbr[g * n + i] : (int32_t)i;
        for (int c0 = 0; c0 < cnt; c0 += G) {
            const int q = c0 + g;
            const bool valid = q < cnt;
            const int64_t slot = i * kmax + q;
            const int32_t j = jn;
            jn = q + G < cnt ? L.nbr[(q + G) * n + i] : (int32_t)i;
            const D4 pj = P[j];
            ContactIn c;
            c.dx = min_image(pi.x - pj.x, s.L[0], s.hL[0], s.periodic[0]);
            c.dy = min_image(pi.y - pj.y, s.L[1], s.hL[1], s.periodic[1]);
            c.dz = min_image(pi.z - pj.z, s.L[2], s.hL[2], s.periodic[2]);
            c.ra = ri;
            c.rb = pj.w;
            const double rs = c.ra + c.rb;
            double fx = 0.0, fy = 0.0, fz = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
            bool hit = false, stored = false;
            if (valid && c.dx * c.dx + c.dy * c.dy + c.dz * c.dz < rs * rs) {
                const D4 vj = V[j];
                const D4 sj = S[j];
                double hx = 0.0, hy = 0.0, hz = 0.0;
                if ((mask >> q) & 1ull) {
                    const D4 h = L.xi[slot];
                    hx = h.x; hy = h.y; hz = h.z;
                }
                c.ma = mi; c.mb = vj.w;
                c.vrx = vi.x - vj.x; c.vry = vi.y - vj.y; c.vrz = vi.z - vj.z;
                c.wsx = ri * si.x + pj.w * sj.x;
                c.wsy = ri * si.y + pj.w * sj.y;
                c.wsz = ri * si.z + pj.w * sj.z;
                const PairCoef pc = coef[ti * s.ntypes + ((int)sj.w & 15)];
                double ftx, fty, ftz, nx, ny, nz, fn;
                if (contact_force(c, false, pc, s.dt, update != 0, hx, hy, hz, fx, fy, fz, ftx, fty, ftz, nx, ny,
                                  nz, fn)) {
                    if (COUNT) ++ncont;
                    hit = true;
                    tx = -(ri * (ny * ftz - nz * fty));
                    ty = -(ri * (nz * ftx - nx * ftz));
                    tz = -(ri * (nx * fty - ny * ftx));
                    if (update) {
                        L.xi[slot] = D4{hx, hy, hz, 0.0};
                        stored = true;
                    }
                }
            }
            // add this chunk's contacts in ascending slot order
            uint64_t b = (__ballot(hit) >> gbase) & gmask;
            while (b) {
                const int src_lane = gbase + __builtin_ctzll(b);
                b &= b - 1;
                Fx = Fx + __shfl(fx, src_lane);
                Fy = Fy + __shfl(fy, src_lane);
                Fz = Fz + __shfl(fz, src_lane);
                Tx = Tx + __shfl(tx, src_lane);
                Ty = Ty + __shfl(ty, src_lane);
                Tz = Tz + __shfl(tz, src_lane);
            }
            nmask |= ((__ballot(stored) >> gbase) & gmask) << c0;
        }
        // the wall (every lane of the group computes it; lane 0 stores)
        if (s.wall && pi.z < ri) {
            ContactIn c;
            c.dx = 0.0; c.dy = 0.0; c.dz = pi.z;
            c.ra = ri; c.rb = 0.0; c.ma = mi; c.mb = 0.0;
            c.vrx = vi.x; c.vry = vi.y; c.vrz = vi.z;
            c.wsx = ri * si.x; c.wsy = ri * si.y; c.wsz = ri * si.z;
            const PairCoef pc = coef[ti * s.ntypes + ti];
            double hx = 0.0, hy = 0.0, hz = 0.0;
            if (mask & kWallBit) { hx = a.xiw[i]; hy = a.xiw[n + i]; hz = a.xiw[2 * n + i]; }
            double fx, fy, fz, ftx, fty, ftz, nx, ny, nz, fn;
            if (contact_force(c, true, pc, s.dt, update != 0, hx, hy, hz, fx, fy, fz, ftx, fty, ftz, nx, ny, nz,
                              fn)) {
                if (COUNT && g == 0) ++nwall;
                Fx = Fx + fx; Fy = Fy + fy; Fz = Fz + fz;
                Tx = Tx + -(ri * (ny * ftz - nz * fty));
                Ty = Ty + -(ri * (nz * ftx - nx * ftz));
                Tz = Tz + -(ri * (nx * fty - ny * ftx));
                if (update) {
                    if (g == 0) { a.xiw[i] = hx; a.xiw[n + i] = hy; a.xiw[2 * n + i] = hz; }
                    nmask |= kWallBit;
                }
            }
        }
        // the system's static surfaces: lane g of the group takes surfaces g, g + G,
        // ..., stores its own histories, and the contributions are added in table
        // order as the neighbour chunks are
        if (SURF && s.nsurf > 0) {
            const uint32_t sm = a.smask[i];
            uint32_t nsm = 0;
            for (int k0 = 0; k0 < s.nsurf; k0 += G) {   // (uniform over the block)
                const int k = k0 + g;
                double fx = 0.0, fy = 0.0, fz = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
                bool hit = false;
                double dist, wnx, wny, wnz;
                const Surf *w = a.surf + s.surf0 + (k < s.nsurf ? k : 0);
                if (k < s.nsurf && w->enabled && surf_gap(*w, pi.x, pi.y, pi.z, ri, dist, wnx, wny, wnz)) {
                    PairCoef pc = coef[ti * s.ntypes + ti];
                    if (w->mu >= 0.0) pc.mu = w->mu;
                    ContactIn c;
                    c.dx = 0.0; c.dy = 0.0; c.dz = dist;
                    c.ra = ri; c.rb = 0.0; c.ma = mi; c.mb = 0.0;
                    c.vrx = vi.x; c.vry = vi.y; c.vrz = vi.z;
                    c.wsx = ri * si.x; c.wsy = ri * si.y; c.wsz = ri * si.z;
                    double hx = 0.0, hy = 0.0, hz = 0.0;
                    if ((sm >> k) & 1u) {
                        const D4 h = a.sxi[k * n + i];
                        hx = h.x; hy = h.y; hz = h.z;
                    }
                    double ftx, fty, ftz, nx, ny, nz, fn;
                    if (contact_force_n(c, true, wnx, wny, wnz, pc, s.dt, update != 0, hx, hy, hz, fx, fy, fz, ftx,
                                        fty, ftz, nx, ny, nz, fn)) {
                        if (COUNT) ++nwall;
                        hit = true;
                        tx = -(ri * (ny * ftz - nz * fty));
                        ty = -(ri * (nz * ftx - nx * ftz));
                        tz = -(ri * (nx * fty - ny * ftx));
                        if (update) a.sxi[k * n + i] = D4{hx, hy, hz, 0.0};
                    }
                }
                uint64_t b = (__ballot(hit) >> gbase) & gmask;
                if (update) nsm |= (uint32_t)b << k0;
                while (b) {
                    const int src_lane = gbase + __builtin_ctzll(b);
                    b &= b - 1;
                    Fx = Fx + __shfl(fx, src_lane);
                    Fy = Fy + __shfl(fy, src_lane);
                    Fz = Fz + __shfl(fz, src_lane);
                    Tx = Tx + __shfl(tx, src_lane);
                    Ty = Ty + __shfl(ty, src_lane);
                    Tz = Tz + __shfl(tz, src_lane);
                }
            }
            if (update && g == 0 && nsm != sm) a.smask[i] = nsm;
        }
        // external force (the coupling's correcting force), added last
        if (a.fext) {
            Fx = Fx + a.fext[i];
            Fy = Fy + a.fext[n + i];
            Fz = Fz + a.fext[2 * n + i];
        }
        if (g != 0) return;
        if (update && nmask != mask) L.mask[i] = nmask;
        if (MODE == 0) {
            a.f[i] = Fx; a.f[n + i] = Fy; a.f[2 * n + i] = Fz;
            a.t[i] = Tx; a.t[n + i] = Ty; a.t[2 * n + i] = Tz;
            return;
        }
        // kick 1/2 with the new forces
        const D2 im = a.im[i];
        double vx = vi.x + s.hdt * (Fx * im.a), vy = vi.y + s.hdt * (Fy * im.a), vz = vi.z + s.hdt * (Fz * im.a);
        double wx = si.x + s.hdt * (Tx * im.b), wy = si.y + s.hdt * (Ty * im.b), wz = si.z + s.hdt * (Tz * im.b);
        if (MODE == 2 || (MR && last)) {
            a.f[i] = Fx; a.f[n + i] = Fy; a.f[2 * n + i] = Fz;
            a.t[i] = Tx; a.t[n + i] = Ty; a.t[2 * n + i] = Tz;
            a.x[i] = pi.x; a.x[n + i] = pi.y; a.x[2 * n + i] = pi.z;
            a.v[i] = vx; a.v[n + i] = vy; a.v[2 * n + i] = vz;
            a.w[i] = wx; a.w[n + i] = wy; a.w[2 * n + i] = wz;
        } else {
            // next step: kick 1/2, drift, wrap, displacement since the last build
            vx = vx + s.hdt * (Fx * im.a); vy = vy + s.hdt * (Fy * im.a); vz = vz + s.hdt * (Fz * im.a);
            wx = wx + s.hdt * (Tx * im.b); wy = wy + s.hdt * (Ty * im.b); wz = wz + s.hdt * (Tz * im.b);
            const double x = wrap_axis(pi.x + s.dt * vx, s, 0);
            const double y = wrap_axis(pi.y + s.dt * vy, s, 1);
            const double z = wrap_axis(pi.z + s.dt * vz, s, 2);
            const double ddx = a.disp[i] + s.dt * vx;
            const double ddy = a.disp[n + i] + s.dt * vy;
            const double ddz = a.disp[2 * n + i] + s.dt * vz;
            a.disp[i] = ddx; a.disp[n + i] = ddy; a.disp[2 * n + i] = ddz;
            double dsq = 0.0;
            dsq += ddx * ddx;
            dsq += ddy * ddy;
            dsq += ddz * ddz;
            if (!(dsq <= s.disp_thr2)) {
                need = true;
                a.sel[sy] = 1;
            }
            if (!isfinite(x + y + z + vx + vy + vz)) bad = true;
            a.pos[src ^ 1][i] = D4{x, y, z, ri};
            a.vel[src ^ 1][i] = D4{vx, vy, vz, mi};
            a.spin[src ^ 1][i] = D4{wx, wy, wz, si.w};
        }
}

template <bool BATCH, bool COUNT, int MODE, int G, bool MR, bool SURF>
// Compiled for four waves per SIMD (at most 128 registers): the kernel waits
// on gathers, and the fourth wave ran the 1e6-sphere bed 15 % and the
// 64-system batch 14 % faster than three (the batch form spills a few bytes
// and still gains); at five or more waves the spills cost more than the
// extra wave brings.
__global__ void __launch_bounds__(256, 4) k_step(KArgs a, int src, int k, int update) {
    int64_t step = 0, cbase = 0, send = 0;
    if (MODE != 0) {
        step = a.flags->step_base + k;
        if (a.flags->abort_at <= step) return;
        update = 1;
        if (MR) {
            cbase = a.flags->call_base;
            send = a.flags->step_end;
        }
    }
    const int g = threadIdx.x % G;
    const int ppb = blockDim.x / G;                        // particles per tile
    const int gbase = (threadIdx.x % warpSize) / G * G;    // first lane of the group in the wave
    const uint64_t gmask = (1ull << G) - 1;
    unsigned ncont = 0, nwall = 0;
    bool need = false, bad = false;
    // a batch is walked in tiles that each lie within one system, so that the
    // block's system descriptor is uniform too; it is read again only when a
    // block moves on to a tile of another system.  Multi-rate: only the tiles of
    // the systems that step at this substep, a prefix of the tiles in stride
    // order, spread over the XCDs like all tiles otherwise
    // tiles over the systems' live particles (the table follows insertions and removals)
    int64_t ntiles = uniform_i64(a.tile0[a.nsys]);
    if (MR) {
        const int64_t q1 = step - cbase - 1;
        const int lvl = q1 == 0 ? kMaxLevels - 1 : min(__builtin_ctzll((unsigned long long)q1), kMaxLevels - 1);
        ntiles = uniform_i64(a.mlevel[lvl]);
    }
    const int64_t *tt0 = MR ? a.mtile0 : a.tile0;
    const int per = gridDim.x / kXcd;
    const int64_t chunk = (ntiles + kXcd - 1) / kXcd;
    const int64_t t0 = (blockIdx.x % kXcd) * chunk;
    const int64_t t1 = t0 + chunk < ntiles ? t0 + chunk : ntiles;
    SysDesc sd = uniform_sys(a.sys);   // the only system when !BATCH
    int sy = 0;
    int64_t tlo = 0, thi = BATCH ? 0 : ntiles;
    // the system's current list (its buffer index changes only between launches)
    int lc = __builtin_amdgcn_readfirstlane(a.lcur[0]);
    if (!BATCH) load_step_coef(a, sd);
    for (int64_t t = t0 + blockIdx.x / kXcd; t < t1; t += per) {   // uniform over the block
        if (BATCH && (t < tlo || t >= thi)) {
            int lo = 0, hi = a.nsys - 1;   // last system (in the tile order) whose first tile is <= t
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (tt0[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            const int k = __builtin_amdgcn_readfirstlane(lo);
            sy = MR ? __builtin_amdgcn_readfirstlane(a.msys[k]) : k;
            sd = uniform_sys(a.sys + sy);
            tlo = uniform_i64(tt0[k]);
            thi = uniform_i64(tt0[k + 1]);
            lc = __builtin_amdgcn_readfirstlane(a.lcur[sy]);
            load_step_coef(a, sd);
        }
        if (BATCH && a.only_sys >= 0 && sy != a.only_sys) continue;   // (uniform over the block)
        int srcs = src;
        bool last = MODE == 2;
        if (MR) {
            // multi-rate: the system steps at substeps 1, 1 + stride, ... of the call
            // (every tile walked here is one of a stepping system); its state
            // alternates between the buffers at its own steps
            const int64_t q1 = step - cbase - 1;
            srcs = (int)((q1 / sd.stride) & 1);
            last = step + sd.stride - 1 == send;
        }
        const int64_t i = BATCH ? sd.p0 + (t - tlo) * ppb + threadIdx.x / G : t * ppb + threadIdx.x / G;
        if (i >= sd.pe) continue;   // past the system's live particles
        const D4 pi = a.pos[srcs][i], vi = a.vel[srcs][i], si = a.spin[srcs][i];
        step_particle<BATCH, COUNT, MODE, G, MR, SURF>(a, sd, (lc & 1) ? a.lst[1] : a.lst[0], srcs, update, i, sy, pi, vi,
                                                 si, (int)si.w, g, gbase, gmask, ncont, nwall, need, bad, last);
    }
    if (bad) atomicOr(&a.flags->err, kErrNonFinite);
    if (MODE == 1 && need) a.flags->abort_at = step + 1;
    // the call's last step ran: count the call's steps (no extra launch and synchronisation)
    if (MODE != 0 && a.call_steps > 0 && blockIdx.x == 0 && threadIdx.x == 0) a.flags->steps += a.call_steps;
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

// ------------------------------------------------------------------ launchers

// Blocks for a particle kernel: one per tile (rounded up to a multiple of the
// XCD count) unless `cap` (> 0) limits the grid, in which case blocks walk
// several tiles of their XCD's chunk.
static int grid_for(int64_t n, int block, int64_t cap = 0) {
    int64_t tiles = (n + block - 1) / block;
    int64_t g = (tiles + kXcd - 1) / kXcd * kXcd;
    if (cap > 0 && g > cap) g = (cap + kXcd - 1) / kXcd * kXcd;
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

hipError_t launch_scan(const int32_t *in, int64_t m, int32_t *partial, int32_t *out, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    k_scan_partial<<<(int)nb, kScanBlock, 0, st>>>(in, m, partial);
    k_scan_top<<<1, kScanBlock, 0, st>>>(partial, nb);
    k_scan_apply<<<(int)nb, kScanBlock, 0, st>>>(in, m, partial, out);
    CHECK_LAUNCH();
}

hipError_t launch_bin(const KArgs &a, int frame_identity, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipError_t e;
    k_zero_selected_cells<<<flat_grid(a.cw1 - a.cw0 + 1, 256), 256, 0, st>>>(a);
    const int64_t nw = a.w1 - a.w0;
    const int g = grid_for(nw, a.block);
    if (a.nsys > 1) k_bin_count<true><<<g, a.block, 0, st>>>(a);
    else k_bin_count<false><<<g, a.block, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_scan(a.cell_count, a.ncell, a.scan_partial, a.cell_start, st)) != hipSuccess) return e;
    if (a.nsys > 1) k_bin_place<true><<<g, a.block, 0, st>>>(a);
    else k_bin_place<false><<<g, a.block, 0, st>>>(a);
    k_cell_sort<<<flat_grid(a.cw1 - a.cw0, 256), 256, 0, st>>>(a);
    k_gather<<<flat_grid(nw, 256), 256, 0, st>>>(a, frame_identity);
    k_scatter_back<<<flat_grid(nw, 256), 256, 0, st>>>(a);
    CHECK_LAUNCH();
}

hipError_t launch_flip(const KArgs &a, hipStream_t st) {
    k_flip<<<1, 64, 0, st>>>(a);
    CHECK_LAUNCH();
}

// (x, y, z, r) of every particle, packed into the binning scratch (free
// between a bin and the next) for the candidate reads of k_neighbors.
__global__ void k_nbr_pack(KArgs a) {
    const int64_t n = a.n;
    D4 *Q = (D4 *)a.shadow_d;
    FOR_WINDOW_FLAT(a, i) Q[i] = D4{a.x[i], a.x[n + i], a.x[2 * n + i], a.r[i]};
}

hipError_t launch_neighbors(const KArgs &a, int have_old, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    k_nbr_pack<<<flat_grid(a.w1 - a.w0, 256), 256, 0, st>>>(a);
    // per-group hit, id and previous-id buffers (24 KB per block at kmax = 32)
    const int block = kNbrBlock;
    const size_t lds = nbr_lds_bytes(a.kmax, block);
    const int g = grid_for((a.w1 - a.w0) * kNbrLanes, block);
    if (a.nsys > 1) k_neighbors<true><<<g, block, lds, st>>>(a, have_old);
    else k_neighbors<false><<<g, block, lds, st>>>(a, have_old);
    CHECK_LAUNCH();
}

hipError_t launch_pack(const KArgs &a, int dst, int mode, int k, int gate, hipStream_t st, int64_t qa) {
    if (a.n <= 0) return hipSuccess;
    const int g = grid_for(a.w1 - a.w0, a.block);
    if (a.nsys > 1) k_pack<true><<<g, a.block, 0, st>>>(a, dst, mode, k, gate, qa);
    else k_pack<false><<<g, a.block, 0, st>>>(a, dst, mode, k, gate, qa);
    CHECK_LAUNCH();
}

hipError_t launch_unpack(const KArgs &a, int src, int selected, hipStream_t st, int64_t qa) {
    if (a.n <= 0) return hipSuccess;
    k_unpack<<<flat_grid(a.w1 - a.w0, 256), 256, 0, st>>>(a, src, selected, qa);
    CHECK_LAUNCH();
}

template <int G>
static hipError_t launch_step_g(const KArgs &a, int src, int mode, int k, int update, int count, hipStream_t st) {
    const int64_t ntiles = a.ntiles_b;
    const int g = grid_for(ntiles * a.block, a.block, a.grid_cap);
    const int B = a.block;
#define STEP_LAUNCH(BT, CT, MD, SF) k_step<BT, CT, MD, G, false, SF><<<g, B, 0, st>>>(a, src, k, update)
#define STEP_MODES(BT, CT, SF)                                  \
    if (mode == 0) STEP_LAUNCH(BT, CT, 0, SF);                  \
    else if (mode == 1) STEP_LAUNCH(BT, CT, 1, SF);             \
    else STEP_LAUNCH(BT, CT, 2, SF)
    if (a.nsys > 1 && a.multirate && mode != 0) {
        // each system decides per block whether the substep is one of its steps
        // and whether it is its last one of the call (the mode-2 epilogue)
        if (a.sxi) {
            if (count) k_step<true, true, 1, G, true, true><<<g, B, 0, st>>>(a, src, k, update);
            else k_step<true, false, 1, G, true, true><<<g, B, 0, st>>>(a, src, k, update);
        } else {
            if (count) k_step<true, true, 1, G, true, false><<<g, B, 0, st>>>(a, src, k, update);
            else k_step<true, false, 1, G, true, false><<<g, B, 0, st>>>(a, src, k, update);
        }
    } else if (a.sxi) {   // surfaces: a separate instantiation keeps the others' registers
        if (a.nsys > 1) {
            if (count) { STEP_MODES(true, true, true); } else { STEP_MODES(true, false, true); }
        } else {
            if (count) { STEP_MODES(false, true, true); } else { STEP_MODES(false, false, true); }
        }
    } else if (a.nsys > 1) {
        if (count) { STEP_MODES(true, true, false); } else { STEP_MODES(true, false, false); }
    } else {
        if (count) { STEP_MODES(false, true, false); } else { STEP_MODES(false, false, false); }
    }
#undef STEP_MODES
#undef STEP_LAUNCH
    return hipGetLastError();
}

hipError_t launch_step(const KArgs &a, int src, int mode, int k, int update, int count, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    switch (a.lanes) {
    case 4: return launch_step_g<4>(a, src, mode, k, update, count, st);
    case 16: return launch_step_g<16>(a, src, mode, k, update, count, st);
    default: return launch_step_g<8>(a, src, mode, k, update, count, st);
    }
}

}  // namespace dem
