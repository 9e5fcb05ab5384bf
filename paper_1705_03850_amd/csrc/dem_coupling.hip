// dem_coupling.hip -- cell fields and coupling controllers of the multi-level
// coarse-grain model (Sec. 2.3, Eq. (7)): kernels and the C-ABI calls
// dem_cell_fields, dem_pi_control, dem_p_control and dem_set_external_force.
//
// Fields: the spheres of a cell are found through the list's binning (the
// particle range of every bin row that the cell, widened by one bin on each
// side, touches: spheres stay within one bin of their binned position until
// the next rebuild).  A cell's bin rows are dealt to S workgroups (S from the
// cell count, so that few large cells still fill the device, and from the
// cell's number of bin rows, so that a slice holds about eight of them); a
// workgroup lays its rows' candidates end to end (a scan of the row lengths
// in LDS) and its threads take them in turn, G threads per sphere where the
// sphere's contacts are summed.  Each thread sums its own terms, the block
// adds the threads' sums in a fixed tree (all sums at once), and one block
// per cell adds the S slices in the same kind of tree: the result depends on
// nothing but the state, the grid, the binning and the workspace size.  A
// first pass gives mass and momentum, hence the Favre velocity; the second
// the kinetic and contact parts of Eq. (7), the contact forces evaluated as
// in a force pass without history update.
// Controllers: one thread per cell updates the PI state; one thread per
// sphere of the system writes its external force.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dem_ctx.h"

namespace dem {
namespace {

struct FGrid {
    double lo[3], h[3];
    int32_t n[3];
    int32_t sys;
    int64_t ncell;
    double vol;   // cell volume h0 h1 h2
};

constexpr int kFB = 256;   // threads per workgroup of the fields kernels

// Coupled stepping (dem_step_coupled) enqueues several intervals at once: a
// kernel given the flag block does nothing while a list rebuild is pending
// (the call issues it again after the rebuild).  Null: always runs.
__device__ inline bool skip_pending(const Flags *gate) { return gate && gate->abort_at != INT64_MAX; }
constexpr int kFG = 4;     // threads per sphere where its contacts are summed

// Cell of a centre: floor((x - lo) / h) per axis, -1 outside (or NaN).
__device__ inline int64_t field_cell(const FGrid &g, double x, double y, double z) {
    const double u0 = floor((x - g.lo[0]) / g.h[0]);
    const double u1 = floor((y - g.lo[1]) / g.h[1]);
    const double u2 = floor((z - g.lo[2]) / g.h[2]);
    if (!(u0 >= 0.0 && u0 < (double)g.n[0] && u1 >= 0.0 && u1 < (double)g.n[1] && u2 >= 0.0 &&
          u2 < (double)g.n[2]))
        return -1;
    return ((int64_t)u2 * g.n[1] + (int64_t)u1) * g.n[0] + (int64_t)u0;
}

// Bins of one axis that a cell [b0, b1) widened by `margin` touches: one or
// two inclusive ranges (two where a periodic axis wraps).  On an open axis the
// range is clamped into the grid (spheres outside it sit in the edge bins).
struct Pieces {
    int s[2], e[2], np;
};

__device__ inline Pieces axis_pieces(const SysDesc &sd, int a, double b0, double b1, double margin) {
    const int nc = sd.nc[a];
    double f0 = floor((b0 - margin - sd.lo[a]) * sd.inv_w[a]);
    double f1 = floor((b1 + margin - sd.lo[a]) * sd.inv_w[a]);
    f0 = fmin(fmax(f0, -1e9), 1e9);
    f1 = fmin(fmax(f1, -1e9), 1e9);
    Pieces p;
    p.np = 1;
    p.s[1] = p.e[1] = 0;
    if (sd.periodic[a]) {
        if (f1 - f0 + 1.0 >= (double)nc) {
            p.s[0] = 0;
            p.e[0] = nc - 1;
            return p;
        }
        int k0 = (int)f0 % nc, k1 = (int)f1 % nc;
        if (k0 < 0) k0 += nc;
        if (k1 < 0) k1 += nc;
        if (k0 <= k1) {
            p.s[0] = k0;
            p.e[0] = k1;
        } else {
            p.s[0] = k0;
            p.e[0] = nc - 1;
            p.s[1] = 0;
            p.e[1] = k1;
            p.np = 2;
        }
    } else {
        p.s[0] = (int)fmin(fmax(f0, 0.0), (double)(nc - 1));
        p.e[0] = (int)fmin(fmax(f1, 0.0), (double)(nc - 1));
    }
    return p;
}

// Sums of N values per thread (the last one a maximum when LASTMAX), each in
// the same fixed tree over the block, all N at once (one barrier per level);
// the results land in v of thread 0.  lds holds N kFB doubles.
template <int N, bool LASTMAX>
__device__ inline void block_reduce_n(double (&v)[N], double *lds) {
    const int t = threadIdx.x;
    __syncthreads();
    for (int k = 0; k < N; ++k) lds[k * kFB + t] = v[k];
    __syncthreads();
    for (int off = kFB / 2; off > 0; off >>= 1) {
        if (t < off)
            for (int k = 0; k < N; ++k) {
                const double a = lds[k * kFB + t], b = lds[k * kFB + t + off];
                lds[k * kFB + t] = (LASTMAX && k == N - 1) ? fmax(a, b) : a + b;
            }
        __syncthreads();
    }
    for (int k = 0; k < N; ++k) v[k] = lds[k * kFB];
}

// The bin rows (bz, by) a cell touches, numbered r = zi * RY + yi over the
// pieces of Z and Y; slice b of S takes rows b, b + S, ...  Calls visit(p) for
// every candidate sphere index p of those rows, the block's threads taking
// them in turn (the same loop bounds in every thread).
__device__ inline int piece_len(const Pieces &P) {
    return (P.e[0] - P.s[0] + 1) + (P.np > 1 ? P.e[1] - P.s[1] + 1 : 0);
}
__device__ inline int piece_at(const Pieces &P, int k) {
    const int l0 = P.e[0] - P.s[0] + 1;
    return k < l0 ? P.s[0] + k : P.s[1] + (k - l0);
}

// Exclusive prefix sum of one int per thread over the block, and the total.
__device__ inline int block_excl_scan(int v, int *wsum, int &total) {
    const int lane = threadIdx.x % warpSize, wid = threadIdx.x / warpSize;
    int x = v;
    for (int o = 1; o < warpSize; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == warpSize - 1) wsum[wid] = x;
    __syncthreads();
    int base = 0;
    total = 0;
    for (int w = 0; w < kFB / warpSize; ++w) {
        if (w < wid) base += wsum[w];
        total += wsum[w];
    }
    __syncthreads();
    return base + x - v;
}

// Candidate list of a workgroup in LDS: each of up to kFB rows gives at most
// two particle ranges (the X pieces); off is their exclusive scan.
struct CandLds {
    int32_t beg[2 * kFB];
    int32_t off[2 * kFB + 1];
    int32_t wsum[kFB / 64];
};

// Calls visit(p, lane) for every candidate sphere p of slice b of S of the
// cell's bin rows (rows b, b + S, ...), G lanes per candidate: the rows are
// taken kFB at a time and their ranges laid end to end; candidate q of such a
// chunk goes to the G threads that start at G (q mod kFB / G), as lanes 0 to
// G - 1.
template <int G, class F>
__device__ inline void for_candidates(const KArgs &a, const SysDesc &sd, const Pieces &X, const Pieces &Y,
                                      const Pieces &Z, int b, int S, CandLds &sh, F visit) {
    const int32_t *cs = a.cell_start;
    const int RY = piece_len(Y), R = piece_len(Z) * RY;
    const int nr = b < R ? (R - b + S - 1) / S : 0;
    const int t = threadIdx.x;
    for (int r0 = 0; r0 < nr; r0 += kFB) {
        int32_t b0 = 0, l0 = 0, b1 = 0, l1 = 0;
        const int k = r0 + t;
        if (k < nr) {
            const int r = b + k * S;
            const int bz = piece_at(Z, r / RY), by = piece_at(Y, r % RY);
            const int64_t row = sd.c0 + ((int64_t)bz * sd.nc[1] + by) * sd.nc[0];
            b0 = cs[row + X.s[0]];
            l0 = cs[row + X.e[0] + 1] - b0;
            if (X.np > 1) {
                b1 = cs[row + X.s[1]];
                l1 = cs[row + X.e[1] + 1] - b1;
            }
        }
        int total;
        const int off = block_excl_scan(l0 + l1, sh.wsum, total);
        sh.beg[2 * t] = b0;
        sh.beg[2 * t + 1] = b1;
        sh.off[2 * t] = off;
        sh.off[2 * t + 1] = off + l0;
        if (t == 0) sh.off[2 * kFB] = total;
        __syncthreads();
        for (int q = t / G; q < total; q += kFB / G) {
            int lo = 0, hi = 2 * kFB;   // the last range that starts at or before q
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sh.off[mid] <= q) lo = mid;
                else hi = mid;
            }
            visit(sh.beg[lo] + (q - sh.off[lo]), t % G);
        }
        __syncthreads();
    }
}

// Sums of one cell's slice: pass 1 (count, mass, momentum, solids volume,
// largest speed), pass 2 (Eq. (7): contact part 1/2 d (x) f over every contact
// of the cell's spheres, kinetic part m v' (x) v' with v' = v - u, u the
// cell's Favre velocity).
constexpr int kP1 = 7, kP2 = 15;

struct CellBox {
    Pieces X, Y, Z;
};

__device__ inline CellBox cell_box(const SysDesc &sd, const FGrid &g, int64_t cell) {
    const int64_t c0 = cell % g.n[0], c1 = (cell / g.n[0]) % g.n[1], c2 = cell / ((int64_t)g.n[0] * g.n[1]);
    const double b0[3] = {g.lo[0] + (double)c0 * g.h[0], g.lo[1] + (double)c1 * g.h[1], g.lo[2] + (double)c2 * g.h[2]};
    CellBox B;
    B.X = axis_pieces(sd, 0, b0[0], b0[0] + g.h[0], 1.0 / sd.inv_w[0]);
    B.Y = axis_pieces(sd, 1, b0[1], b0[1] + g.h[1], 1.0 / sd.inv_w[1]);
    B.Z = axis_pieces(sd, 2, b0[2], b0[2] + g.h[2], 1.0 / sd.inv_w[2]);
    return B;
}

// Every sphere of the system must lie within one bin width (per axis) of its
// position at the last list build for the bin-row search to find it: blocks
// `blk` of `nblk` check a share of the system's spheres.
__device__ inline void fields_guard(const KArgs &a, int32_t sys, int64_t blk, int64_t nblk) {
    const SysDesc &sd = a.sys[sys];
    const int64_t n = a.n;
    bool bad = false;
    for (int64_t i = sd.p0 + blk * blockDim.x + threadIdx.x; i < sd.pe; i += nblk * blockDim.x)
        for (int ax = 0; ax < 3; ++ax)
            if (!(fabs(a.disp[ax * n + i]) * sd.inv_w[ax] <= 1.0)) bad = true;
    if (bad) atomicOr(&a.flags->err, kErrStale);
}

// Block (cell, b): slice b of S of the cell's rows.  S = 1 writes the cell's
// rows of `out` directly; S > 1 writes the slice's sums to part[(cell S + b) kP1].
// The blocks after the ncell S field blocks run the guard above.
__global__ void __launch_bounds__(kFB) k_fields1(KArgs a, FGrid g, int S, double *part, double *out,
                                                 const Flags *gate) {
    __shared__ double lds[kP1 * kFB];
    __shared__ CandLds sh;
    if (skip_pending(gate)) return;
    const int64_t nfb = g.ncell * S;
    if ((int64_t)blockIdx.x >= nfb) {
        fields_guard(a, g.sys, (int64_t)blockIdx.x - nfb, (int64_t)gridDim.x - nfb);
        return;
    }
    const SysDesc sd = a.sys[g.sys];
    const int64_t n = a.n;
    const int64_t cell = blockIdx.x / S;
    const int b = blockIdx.x % S;
    const CellBox B = cell_box(sd, g, cell);
    double cnt = 0.0, mass = 0.0, px = 0.0, py = 0.0, pz = 0.0, vol = 0.0, vmax = 0.0;
    for_candidates<1>(a, sd, B.X, B.Y, B.Z, b, S, sh, [&](int32_t i, int) {
        if (field_cell(g, a.x[i], a.x[n + i], a.x[2 * n + i]) != cell) return;
        const double m = a.m[i], r = a.r[i];
        const double vx = a.v[i], vy = a.v[n + i], vz = a.v[2 * n + i];
        cnt += 1.0;
        mass += m;
        px += m * vx;
        py += m * vy;
        pz += m * vz;
        vol += 4.0 / 3.0 * M_PI * r * r * r;
        vmax = fmax(vmax, sqrt(vx * vx + vy * vy + vz * vz));
    });
    double v[kP1] = {cnt, mass, px, py, pz, vol, vmax};
    block_reduce_n<kP1, true>(v, lds);
    if (threadIdx.x == 0) {
        if (S == 1) {
            const int64_t nc = g.ncell;
            const int rows[kP1] = {DEM_F_COUNT, DEM_F_MASS, DEM_F_MOM, DEM_F_MOM + 1, DEM_F_MOM + 2, DEM_F_VOLUME,
                                   DEM_F_VMAX};
            for (int k = 0; k < kP1; ++k) out[rows[k] * nc + cell] = v[k];
        } else {
            for (int k = 0; k < kP1; ++k) part[(cell * S + b) * kP1 + k] = v[k];
        }
    }
}

// A cell's pass-1 sums over its S <= kFB slices, taken by a whole block:
// thread t loads slice t (zeros past S), then the block's fixed tree (the
// maximum for the last); every thread gets the totals.  The same routine
// wherever the totals are taken, so they agree bit for bit.
__device__ inline void block_pass1_total(const double *part, int64_t cell, int S, double (&v)[kP1], double *lds) {
    const int t = threadIdx.x;
    for (int k = 0; k < kP1; ++k) v[k] = t < S ? part[(cell * S + t) * kP1 + k] : 0.0;
    block_reduce_n<kP1, true>(v, lds);
}

__device__ inline void write_pass1(double *out, int64_t nc, int64_t cell, const double (&v)[kP1]) {
    const int rows[kP1] = {DEM_F_COUNT, DEM_F_MASS, DEM_F_MOM, DEM_F_MOM + 1, DEM_F_MOM + 2, DEM_F_VOLUME, DEM_F_VMAX};
    for (int k = 0; k < kP1; ++k) out[rows[k] * nc + cell] = v[k];
}

// One block per cell (the fields without stress): the slices' sums.
__global__ void __launch_bounds__(kFB) k_fields1_reduce(FGrid g, int S, const double *part, double *out,
                                                        const Flags *gate) {
    __shared__ double lds[kP1 * kFB];
    if (skip_pending(gate)) return;
    const int64_t nc = g.ncell;
    for (int64_t cell = blockIdx.x; cell < nc; cell += gridDim.x) {   // (uniform over the block)
        double v[kP1];
        block_pass1_total(part, cell, S, v, lds);
        if (threadIdx.x == 0) write_pass1(out, nc, cell, v);
    }
}

// Pass 2.  S > 1: the cell's pass-1 totals are taken from the slices in
// part1 by every block of the cell (block 0 also writes them to `out`), and
// the slice's pass-2 sums go to part2[(cell S + b) kP2].
__global__ void __launch_bounds__(kFB) k_fields2(KArgs a, FGrid g, int S, const double *part1, double *part2,
                                                 double *out, const Flags *gate) {
    __shared__ double lds[kP2 * kFB];
    __shared__ CandLds sh;
    if (skip_pending(gate)) return;
    const SysDesc sd = a.sys[g.sys];
    const int64_t n = a.n;
    const int64_t nc = g.ncell;
    const int64_t cell = blockIdx.x / S;
    const int b = blockIdx.x % S;
    if (cell >= nc) return;
    const List L = (a.lcur[g.sys] & 1) ? a.lst[1] : a.lst[0];
    const int64_t kmax = a.kmax;
    const PairCoef *coef = a.coef + sd.coef0;
    const CellBox B = cell_box(sd, g, cell);
    // the cell's Favre velocity from pass 1
    double p1[kP1];
    if (S > 1) {
        block_pass1_total(part1, cell, S, p1, lds);
        if (b == 0 && threadIdx.x == 0) write_pass1(out, nc, cell, p1);
    } else {
        p1[1] = out[DEM_F_MASS * nc + cell];
        for (int k = 0; k < 3; ++k) p1[2 + k] = out[(DEM_F_MOM + k) * nc + cell];
    }
    const double mass = p1[1];
    double ux = 0.0, uy = 0.0, uz = 0.0;
    if (mass > 0.0) {
        ux = p1[2] / mass;
        uy = p1[3] / mass;
        uz = p1[4] / mass;
    }
    double con[9], kin[6];
    for (int k = 0; k < 9; ++k) con[k] = 0.0;
    for (int k = 0; k < 6; ++k) kin[k] = 0.0;
    for_candidates<kFG>(a, sd, B.X, B.Y, B.Z, b, S, sh, [&](int32_t i, int lane) {
        const double xi = a.x[i], yi = a.x[n + i], zi = a.x[2 * n + i];
        if (field_cell(g, xi, yi, zi) != cell) return;
        const double m = a.m[i], ri = a.r[i];
        const double vx = a.v[i], vy = a.v[n + i], vz = a.v[2 * n + i];
        const double wx = a.w[i], wy = a.w[n + i], wz = a.w[2 * n + i];
        if (lane == 0) {
            const double qx = vx - ux, qy = vy - uy, qz = vz - uz;
            kin[0] += m * qx * qx;
            kin[1] += m * qx * qy;
            kin[2] += m * qx * qz;
            kin[3] += m * qy * qy;
            kin[4] += m * qy * qz;
            kin[5] += m * qz * qz;
        }
        const int ti = a.type[i];
        const int rowlen = L.cnt[i];
        const uint64_t mask = L.mask[i];
        for (int q = lane; q < rowlen; q += kFG) {
            const int32_t j = L.nbr[q * n + i];
            ContactIn c;
            c.dx = min_image(xi - a.x[j], sd.L[0], sd.hL[0], sd.periodic[0]);
            c.dy = min_image(yi - a.x[n + j], sd.L[1], sd.hL[1], sd.periodic[1]);
            c.dz = min_image(zi - a.x[2 * n + j], sd.L[2], sd.hL[2], sd.periodic[2]);
            c.ra = ri;
            c.rb = a.r[j];
            c.ma = m;
            c.mb = a.m[j];
            c.vrx = vx - a.v[j];
            c.vry = vy - a.v[n + j];
            c.vrz = vz - a.v[2 * n + j];
            c.wsx = ri * wx + c.rb * a.w[j];
            c.wsy = ri * wy + c.rb * a.w[n + j];
            c.wsz = ri * wz + c.rb * a.w[2 * n + j];
            double hx = 0.0, hy = 0.0, hz = 0.0;
            if ((mask >> q) & 1ull) {
                const D4 h = L.xi[i * kmax + q];
                hx = h.x; hy = h.y; hz = h.z;
            }
            double fx, fy, fz, ftx, fty, ftz, nx, ny, nz, fn;
            if (!contact_force(c, false, coef[ti * sd.ntypes + a.type[j]], sd.dt, false, hx, hy, hz, fx, fy, fz, ftx,
                               fty, ftz, nx, ny, nz, fn))
                continue;
            const double d[3] = {0.5 * c.dx, 0.5 * c.dy, 0.5 * c.dz};
            const double f[3] = {fx, fy, fz};
            for (int p = 0; p < 3; ++p)
                for (int q2 = 0; q2 < 3; ++q2) con[3 * p + q2] += d[p] * f[q2];
        }
    });
    double v[kP2];
    for (int k = 0; k < 9; ++k) v[k] = con[k];
    for (int k = 0; k < 6; ++k) v[9 + k] = kin[k];
    block_reduce_n<kP2, false>(v, lds);
    if (threadIdx.x == 0) {
        if (S == 1) {
            // kinetic part: symmetric (m q_a q_b = m q_b q_a exactly)
            const int ksym[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
            for (int k = 0; k < 9; ++k) out[(DEM_F_STRESS + k) * nc + cell] = (v[k] + v[9 + ksym[k]]) / g.vol;
        } else {
            for (int k = 0; k < kP2; ++k) part2[(cell * S + b) * kP2 + k] = v[k];
        }
    }
}

__global__ void __launch_bounds__(kFB) k_fields2_reduce(FGrid g, int S, const double *part, double *out,
                                                        const Flags *gate) {
    __shared__ double lds[kP2 * kFB];
    if (skip_pending(gate)) return;
    const int64_t nc = g.ncell;
    const int ksym[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    const int t = threadIdx.x;
    for (int64_t cell = blockIdx.x; cell < nc; cell += gridDim.x) {   // (uniform over the block)
        // one block per cell: thread t loads slice t (S <= kFB), then the fixed tree
        double v[kP2];
        for (int k = 0; k < kP2; ++k) v[k] = t < S ? part[(cell * S + t) * kP2 + k] : 0.0;
        block_reduce_n<kP2, false>(v, lds);
        if (t == 0)
            for (int k = 0; k < 9; ++k) out[(DEM_F_STRESS + k) * nc + cell] = (v[k] + v[9 + ksym[k]]) / g.vol;
    }
}


// PI update per transition cell: e = n.sigma_coarse.n - n.sigma_fine.n,
// integral += e interval, u = kp e + ki integral.
__global__ void k_pi_cells(FGrid g, const double *fine, const double *coarse, double nx, double ny, double nz,
                           double kp, double ki, double interval, double *integral, double *u, const Flags *gate) {
    if (skip_pending(gate)) return;
    const int64_t nc = g.ncell;
    const double nn[3] = {nx, ny, nz};
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        double sf = 0.0, sc = 0.0;
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
                sf += nn[p] * fine[(DEM_F_STRESS + 3 * p + q) * nc + c] * nn[q];
                sc += nn[p] * coarse[(DEM_F_STRESS + 3 * p + q) * nc + c] * nn[q];
            }
        const double e = sc - sf;
        const double I = integral[c] + e * interval;
        integral[c] = I;
        u[c] = kp * e + ki * I;
    }
}

// Correcting force on every sphere of the fine system: u pi r^2 w along the
// inward normal in a transition cell (fade w over `fade` diameters below the
// face), limited by the coarse cell's largest speed; zero elsewhere.
__global__ void k_pi_particles(KArgs a, FGrid g, const double *coarse, const double *u, double nx, double ny,
                               double nz, double face, double fade, const Flags *gate) {
    if (skip_pending(gate)) return;
    const SysDesc &sd = a.sys[g.sys];
    const int64_t n = a.n;
    if (a.flags->err & kErrStale) return;   // fields from a stale list: forces left as they are
    for (int64_t i = sd.p0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < sd.pe;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = a.x[i], y = a.x[n + i], z = a.x[2 * n + i];
        const int64_t c = field_cell(g, x, y, z);
        double mag = 0.0;
        if (c >= 0) {
            const double r = a.r[i];
            const double depth = (x * nx + y * ny + z * nz) - face;
            const double reach = fade * 2.0 * r;
            double w = -1.0;
            if (depth < 0.0) w = 1.0;
            else if (depth < reach) w = 1.0 - depth / reach;
            if (w >= 0.0) {
                mag = u[c] * M_PI * (r * r) * w;
                const double vn = a.v[i] * nx + a.v[n + i] * ny + a.v[2 * n + i] * nz;
                const double vm = coarse[DEM_F_VMAX * g.ncell + c];
                const double m = a.m[i];
                if (mag > 0.0) mag = fmin(mag, fmax(0.0, m * (vm - vn) / sd.dt));
                else if (mag < 0.0) mag = fmax(mag, fmin(0.0, m * (-vm - vn) / sd.dt));
            }
        }
        a.fext_ws[i] = mag * nx;
        a.fext_ws[n + i] = mag * ny;
        a.fext_ws[2 * n + i] = mag * nz;
    }
}

// P controller force on every sphere of the coarse system: kp m (target - u_c)
// in a cell where both levels hold mass, zero elsewhere.
__global__ void k_p_particles(KArgs a, FGrid g, const double *fine, const double *coarse, double kp, int mass_flow,
                              const Flags *gate) {
    if (skip_pending(gate)) return;
    const SysDesc &sd = a.sys[g.sys];
    const int64_t n = a.n, nc = g.ncell;
    if (a.flags->err & kErrStale) return;   // fields from a stale list: forces left as they are
    for (int64_t i = sd.p0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < sd.pe;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = field_cell(g, a.x[i], a.x[n + i], a.x[2 * n + i]);
        double F[3] = {0.0, 0.0, 0.0};
        if (c >= 0) {
            const double mf = fine[DEM_F_MASS * nc + c], mc = coarse[DEM_F_MASS * nc + c];
            if (mf > 0.0 && mc > 0.0) {
                const double ratio = mass_flow ? fine[DEM_F_VOLUME * nc + c] / coarse[DEM_F_VOLUME * nc + c] : 1.0;
                const double m = a.m[i];
                for (int k = 0; k < 3; ++k) {
                    const double target = fine[(DEM_F_MOM + k) * nc + c] / mf * ratio;
                    const double uc = coarse[(DEM_F_MOM + k) * nc + c] / mc;
                    F[k] = kp * m * (target - uc);
                }
            }
        }
        a.fext_ws[i] = F[0];
        a.fext_ws[n + i] = F[1];
        a.fext_ws[2 * n + i] = F[2];
    }
}

// sum += add over m values (the running sum of a fields array).
__global__ void k_fields_add(double *sum, const double *add, int64_t m, const Flags *gate) {
    if (skip_pending(gate)) return;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
        sum[k] += add[k];
}

int grid_blocks(int64_t work, int block) {
    int64_t b = (work + block - 1) / block;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace
}  // namespace dem

using namespace dem;
using namespace dem::host;

namespace {

int make_fgrid(dem_ctx *c, const dem_grid *g, FGrid &out) {
    if (!g) return fail(c, DEM_ERR_ARG, "grid is NULL");
    if (g->sys < 0 || g->sys >= (int32_t)c->geo.sys.size()) return fail(c, DEM_ERR_ARG, "grid.sys out of range");
    int64_t nc = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(g->h[a] > 0.0) || !std::isfinite(g->h[a]) || !std::isfinite(g->lo[a]))
            return fail(c, DEM_ERR_ARG, "grid needs finite lo and h > 0");
        if (g->n[a] < 1) return fail(c, DEM_ERR_ARG, "grid needs n >= 1 on every axis");
        nc *= g->n[a];
        if (nc > (1 << 24)) return fail(c, DEM_ERR_ARG, "grid has more than 2^24 cells");
    }
    memset(&out, 0, sizeof out);
    for (int a = 0; a < 3; ++a) {
        out.lo[a] = g->lo[a];
        out.h[a] = g->h[a];
        out.n[a] = g->n[a];
    }
    out.sys = g->sys;
    out.ncell = nc;
    out.vol = g->h[0] * g->h[1] * g->h[2];
    return DEM_OK;
}

// First use: external forces of every system start at zero.
int enable_fext(dem_ctx *c, const KArgs &a) {
    if (c->fext_on) return DEM_OK;
    HIPCALL(c, launch_fill_f64(a.fext_ws, 3 * c->geo.n, 0.0, c->stream));
    c->fext_on = true;
    return DEM_OK;
}

int pi_control(dem_ctx *c, const dem_state *s, const dem_pi_params *p, const double *fine, const double *coarse,
               double *integral, double *u, const Flags *gate) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!p) return fail(c, DEM_ERR_ARG, "params is NULL");
    FGrid g;
    if ((rc = make_fgrid(c, &p->grid, g))) return rc;
    if (!fine || !coarse || !integral || !u) return fail(c, DEM_ERR_ARG, "a fields or controller array is NULL");
    const double nn = p->nrm[0] * p->nrm[0] + p->nrm[1] * p->nrm[1] + p->nrm[2] * p->nrm[2];
    if (!(std::fabs(nn - 1.0) < 1e-12)) return fail(c, DEM_ERR_ARG, "nrm must be a unit vector");
    if (!(p->fade >= 0.0) || !(p->interval >= 0.0) || !std::isfinite(p->kp) || !std::isfinite(p->ki) ||
        !std::isfinite(p->face))
        return fail(c, DEM_ERR_ARG, "need fade >= 0, interval >= 0 and finite gains and face");
    KArgs a = kargs(c, s);
    if ((rc = enable_fext(c, a))) return rc;
    a = kargs(c, s);
    k_pi_cells<<<grid_blocks(g.ncell, 256), 256, 0, c->stream>>>(g, fine, coarse, p->nrm[0], p->nrm[1], p->nrm[2],
                                                                  p->kp, p->ki, p->interval, integral, u, gate);
    const SysDesc &sd = c->geo.sys[g.sys];
    k_pi_particles<<<grid_blocks(sd.pe - sd.p0, 256), 256, 0, c->stream>>>(a, g, coarse, u, p->nrm[0], p->nrm[1],
                                                                          p->nrm[2], p->face, p->fade, gate);
    HIPCALL(c, hipGetLastError());
    return DEM_OK;
}

int p_control(dem_ctx *c, const dem_state *s, const dem_p_params *p, const double *fine, const double *coarse,
              const Flags *gate) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!p) return fail(c, DEM_ERR_ARG, "params is NULL");
    FGrid g;
    if ((rc = make_fgrid(c, &p->grid, g))) return rc;
    if (!fine || !coarse) return fail(c, DEM_ERR_ARG, "a fields array is NULL");
    if (!std::isfinite(p->kp)) return fail(c, DEM_ERR_ARG, "kp must be finite");
    KArgs a = kargs(c, s);
    if ((rc = enable_fext(c, a))) return rc;
    a = kargs(c, s);
    const SysDesc &sd = c->geo.sys[g.sys];
    k_p_particles<<<grid_blocks(sd.pe - sd.p0, 256), 256, 0, c->stream>>>(a, g, fine, coarse, p->kp,
                                                                         p->mass_flow ? 1 : 0, gate);
    HIPCALL(c, hipGetLastError());
    return DEM_OK;
}

// Both field calls: pass 1 with the guard in the same launch; with `stress`
// pass 2, which also completes pass 1 (S > 1), then the pass-2 slices.
int cell_fields(dem_ctx *c, const dem_state *s, const dem_grid *grid, double *fields, bool stress,
                const Flags *gate = nullptr) {
    int rc = check_state(c, s);
    if (rc) return rc;
    FGrid g;
    if ((rc = make_fgrid(c, grid, g))) return rc;
    if (!fields) return fail(c, DEM_ERR_ARG, "fields is NULL");
    if (!c->list_current) return fail(c, DEM_ERR_STATE, "the cell fields need a neighbour list for the current order");
    KArgs a = kargs(c, s);
    HIPCALL(c, hipGetLastError());
    const SysDesc &sd = c->geo.sys[g.sys];
    // slices per cell: about eight bin rows each (a row of bins holds some tens
    // of candidates), but no more than 4096 workgroups in all (a function of
    // the grid, the system's binning and the workspace only, so the sums'
    // order is too); S = 1 writes the fields directly
    const size_t scratch = (size_t)kShadowD * c->geo.n * 8;
    int64_t rows = 1;
    for (int ax = 1; ax < 3; ++ax) {
        const double w = sd.L[ax] / (double)sd.nc[ax];
        rows *= std::min<int64_t>(sd.nc[ax], (int64_t)std::floor(g.h[ax] / w) + 3);
    }
    int S = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(kFB, 4096 / g.ncell), rows / 8));
    while (S > 1 && (size_t)g.ncell * S * (kP1 + kP2) * 8 > scratch) S /= 2;
    double *part1 = (double *)(c->ws + c->lay.shadow_d);
    double *part2 = part1 + (size_t)g.ncell * S * kP1;
    const int64_t blocks = g.ncell * S, guard = grid_blocks(sd.pe - sd.p0, 256);
    const int reduce_blocks = (int)std::min<int64_t>(g.ncell, 4096);   // one per cell, looping beyond
    if (blocks + guard > INT32_MAX) return fail(c, DEM_ERR_ARG, "grid too large");
    k_fields1<<<(int)(blocks + guard), kFB, 0, c->stream>>>(a, g, S, part1, fields, gate);
    if (stress) {
        k_fields2<<<(int)blocks, kFB, 0, c->stream>>>(a, g, S, part1, part2, fields, gate);
        if (S > 1) k_fields2_reduce<<<reduce_blocks, kFB, 0, c->stream>>>(g, S, part2, fields, gate);
    } else if (S > 1) {
        k_fields1_reduce<<<reduce_blocks, kFB, 0, c->stream>>>(g, S, part1, fields, gate);
    }
    HIPCALL(c, hipGetLastError());
    return DEM_OK;
}

// One interval's coupling calls of a plan, gated by the flag block.
int couple(dem_ctx *c, const dem_state *s, const dem_coupling_plan *p, const dem_grid &pi_set, const dem_grid &p_tgt,
           const Flags *gate) {
    int rc;
    if ((rc = cell_fields(c, s, &p->pi.grid, p->pi_fine, true, gate)) ||
        (rc = cell_fields(c, s, &pi_set, p->pi_coarse, true, gate)) ||
        (rc = pi_control(c, s, &p->pi, p->pi_fine, p->pi_coarse, p->integral, p->u, gate)) ||
        (rc = cell_fields(c, s, &p_tgt, p->p_fine, false, gate)) ||
        (rc = cell_fields(c, s, &p->p.grid, p->p_coarse, false, gate)) ||
        (rc = p_control(c, s, &p->p, p->p_fine, p->p_coarse, gate)))
        return rc;
    if (p->sum) {
        FGrid g;
        if ((rc = make_fgrid(c, &p->sum_grid, g))) return rc;
        if ((rc = cell_fields(c, s, &p->sum_grid, p->sum_tmp, false, gate))) return rc;
        const int64_t m = (int64_t)DEM_F_STRESS * g.ncell;   // the rows without stress
        k_fields_add<<<grid_blocks(m, 256), 256, 0, c->stream>>>(p->sum, p->sum_tmp, m, gate);
        HIPCALL(c, hipGetLastError());
    }
    return DEM_OK;
}

// The plan's grids and parameters, checked once before anything is enqueued.
int plan_ok(dem_ctx *c, const dem_coupling_plan *p, dem_grid &pi_set, dem_grid &p_tgt) {
    if (p->interval_steps < 1 || p->group < 1) return fail(c, DEM_ERR_ARG, "need interval_steps >= 1 and group >= 1");
    if (!p->pi_fine || !p->pi_coarse || !p->p_fine || !p->p_coarse || !p->integral || !p->u)
        return fail(c, DEM_ERR_ARG, "a fields or controller array of the plan is NULL");
    if (p->sum && !p->sum_tmp) return fail(c, DEM_ERR_ARG, "sum needs sum_tmp");
    pi_set = p->pi.grid;
    pi_set.sys = p->pi_setpoint_sys;
    p_tgt = p->p.grid;
    p_tgt.sys = p->p_target_sys;
    FGrid g;
    int rc;
    if ((rc = make_fgrid(c, &p->pi.grid, g)) || (rc = make_fgrid(c, &pi_set, g)) ||
        (rc = make_fgrid(c, &p->p.grid, g)) || (rc = make_fgrid(c, &p_tgt, g)) ||
        (p->sum && (rc = make_fgrid(c, &p->sum_grid, g))))
        return rc;
    const dem_pi_params &q = p->pi;
    const double nn = q.nrm[0] * q.nrm[0] + q.nrm[1] * q.nrm[1] + q.nrm[2] * q.nrm[2];
    if (!(std::fabs(nn - 1.0) < 1e-12)) return fail(c, DEM_ERR_ARG, "nrm must be a unit vector");
    if (!(q.fade >= 0.0) || !(q.interval >= 0.0) || !std::isfinite(q.kp) || !std::isfinite(q.ki) ||
        !std::isfinite(q.face))
        return fail(c, DEM_ERR_ARG, "need fade >= 0, interval >= 0 and finite gains and face");
    if (!std::isfinite(p->p.kp)) return fail(c, DEM_ERR_ARG, "kp must be finite");
    if (c->multirate && p->interval_steps % c->max_stride)
        return fail(c, DEM_ERR_ARG, "multi-rate stepping needs interval_steps to be a multiple of the largest stride");
    return DEM_OK;
}

// The kernels of one coupled interval, in stream order: the coupling, the
// first kick and drift from the caller's arrays, the interval's steps (the
// last writes the caller's arrays), then the step base advanced by the
// interval, so that the same sequence serves every interval of a group.
int enqueue_interval(dem_ctx *c, const dem_state *s, const dem_coupling_plan *p, const dem_grid &pi_set,
                     const dem_grid &p_tgt) {
    int rc;
    const Flags *gate = c->d_flags;
    if ((rc = couple(c, s, p, pi_set, p_tgt, gate))) return rc;
    const KArgs a = kargs(c, s);
    const int64_t I = p->interval_steps;
    HIPCALL(c, launch_pack(a, 0, 1, 0, 1, c->stream));
    for (int64_t q = 1; q <= I; ++q) {
        KArgs al = a;
        if (q == I) al.call_steps = I;
        HIPCALL(c, launch_step(al, (int)((q - 1) & 1), q == I ? 2 : 1, (int)(q - 1), 1, c->count ? 1 : 0,
                               c->stream));
    }
    HIPCALL(c, launch_ctrl(c->d_flags, 1, I, c->stream));
    return DEM_OK;
}

// The interval as one graph, captured again when the plan or the context's
// stepping options changed.  Everything that changes between intervals
// (positions, lists, live counts, tiles, surfaces) is read from the device.
int interval_graph(dem_ctx *c, const dem_state *s, const dem_coupling_plan *p, const dem_grid &pi_set,
                   const dem_grid &p_tgt) {
    std::vector<char> key(sizeof(dem_coupling_plan) + sizeof(dem_state) + 7 * sizeof(void *));
    char *k = key.data();
    memcpy(k, p, sizeof(dem_coupling_plan));
    k += sizeof(dem_coupling_plan);
    memcpy(k, s, sizeof(dem_state));
    k += sizeof(dem_state);
    // the launch shape too: the step kernels' lanes, block and grid cap must
    // match the tile tables that dem_set_launch uploads
    const void *more[7] = {c->ws, c->fext_on ? (const void *)c->lay.fext : nullptr,
                           (const void *)(intptr_t)(c->multirate ? 1 : 0), (const void *)(intptr_t)(c->count ? 1 : 0),
                           (const void *)(intptr_t)c->lanes, (const void *)(intptr_t)c->geo.block,
                           (const void *)(intptr_t)c->grid_cap};
    memcpy(k, more, sizeof more);
    if (c->cpl_exec && key == c->cpl_key) return DEM_OK;
    if (c->cpl_exec) {
        (void)hipGraphExecDestroy(c->cpl_exec);
        c->cpl_exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    HIPCALL(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_interval(c, s, p, pi_set, p_tgt);
    const hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
    const hipError_t e3 = hipGraphInstantiate(&c->cpl_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
        c->cpl_exec = nullptr;
        return hip_fail(c, e3, "hipGraphInstantiate");
    }
    c->cpl_key = key;
    return DEM_OK;
}

}  // namespace

extern "C" {

int dem_cell_fields(dem_ctx *c, const dem_state *s, const dem_grid *grid, double *fields) {
    return cell_fields(c, s, grid, fields, true);
}

int dem_cell_mass_fields(dem_ctx *c, const dem_state *s, const dem_grid *grid, double *fields) {
    return cell_fields(c, s, grid, fields, false);
}

int dem_pi_control(dem_ctx *c, const dem_state *s, const dem_pi_params *p, const double *fine, const double *coarse,
                   double *integral, double *u) {
    return pi_control(c, s, p, fine, coarse, integral, u, nullptr);
}

int dem_p_control(dem_ctx *c, const dem_state *s, const dem_p_params *p, const double *fine, const double *coarse) {
    return p_control(c, s, p, fine, coarse, nullptr);
}

int dem_step_coupled(dem_ctx *c, const dem_state *s, int64_t nintervals, const dem_coupling_plan *plan) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!plan) return fail(c, DEM_ERR_ARG, "plan is NULL");
    if (nintervals < 0) return fail(c, DEM_ERR_ARG, "nintervals < 0");
    dem_grid pi_set, p_tgt;
    if ((rc = plan_ok(c, plan, pi_set, p_tgt))) return rc;
    if (!c->masses) return fail(c, DEM_ERR_STATE, "dem_reset first");
    if (!c->forces_valid)
        return fail(c, DEM_ERR_STATE,
                    "dem_step_coupled needs the forces of the current state: call dem_forces(ctx, s, 0) or "
                    "dem_declare_forces");
    if (nintervals == 0 || c->geo.n == 0) return DEM_OK;
    if (!c->list_current)
        if ((rc = do_bin(c, s, true)) || (rc = do_neighbors(c, s))) return rc;
    {
        KArgs a = kargs(c, s);
        if ((rc = enable_fext(c, a))) return rc;
    }
    const int64_t I = plan->interval_steps;
    Flags h;
    int64_t done = 0;
    while (done < nintervals) {
        // a group of intervals, enqueued together; steps numbered from base + 1
        const int64_t G = std::min<int64_t>(plan->group, nintervals - done);
        const int64_t base = c->step_counter;
        if (c->use_graph && !c->timing && (rc = interval_graph(c, s, plan, pi_set, p_tgt))) return rc;
        HIPCALL(c, launch_ctrl(c->d_flags, 0, base + 1, c->stream));
        for (int64_t j = 0; j < G; ++j) {
            if (c->multirate) {
                HIPCALL(c, launch_ctrl(c->d_flags, 5, base + I * j, c->stream));
                HIPCALL(c, launch_ctrl(c->d_flags, 6, base + I * (j + 1), c->stream));
            }
            if (c->use_graph && !c->timing) HIPCALL(c, hipGraphLaunch(c->cpl_exec, c->stream));
            else if ((rc = enqueue_interval(c, s, plan, pi_set, p_tgt))) return rc;
        }
        if ((rc = read_flags(c, h)) || (rc = collect_times(c)) || (rc = flag_error(c, h))) return rc;
        if (h.abort_at == INT64_MAX) {
            note_steps(c, G * I);
            c->step_counter = base + G * I;
            done += G;
            continue;
        }
        // the drift into step qa of interval jr asked for a new list; every
        // later kernel of the group did nothing: rebuild, finish interval jr
        // as dem_step would, and issue the rest again
        const int64_t qg = h.abort_at - base;
        const int64_t jr = (qg - 1) / I, qa = qg - jr * I, bj = base + jr * I;
        if ((rc = rebuild_at(c, s, qa))) return rc;
        note_rebuild(c, qg - 1);
        HIPCALL(c, launch_ctrl(c->d_flags, 0, bj + qa, c->stream));
        if (c->multirate) {
            HIPCALL(c, launch_ctrl(c->d_flags, 5, bj, c->stream));
            HIPCALL(c, launch_ctrl(c->d_flags, 6, bj + I, c->stream));
        }
        if ((rc = step_loop(c, s, I, bj, qa, h)) || (rc = collect_times(c)) || (rc = flag_error(c, h))) return rc;
        c->step_counter = bj + I;
        done += jr + 1;
    }
    c->binned = false;
    c->forces_valid = true;
    return DEM_OK;
}

int dem_set_external_force(dem_ctx *c, const dem_state *s, const double *fext) {
    int rc = check_state(c, s);
    if (rc) return rc;
    if (!fext) {
        c->fext_on = false;
        return DEM_OK;
    }
    KArgs a = kargs(c, s);
    if (c->geo.n > 0)
        HIPCALL(c, hipMemcpyAsync(a.fext_ws, fext, 3 * (size_t)c->geo.n * sizeof(double), hipMemcpyDeviceToDevice,
                                  c->stream));
    c->fext_on = true;
    return DEM_OK;
}

}  // extern "C"
