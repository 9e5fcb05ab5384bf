// dem_core.h -- device-side data layout and per-contact arithmetic of the
// DEM contact pipeline (gfx950).  Included by the kernel and the host
// translation units of libdem.so only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dem {

constexpr int kMaxTypes = 4;
constexpr int kMaxSlots = 63;           // neighbour slots per particle (bit 63 of a mask = wall)
constexpr int kCellSortMax = 64;        // cells holding more particles are left unsorted (flagged)
constexpr uint64_t kWallBit = 1ull << 63;

// Sticky error bits of the device flag block.
enum : int { kErrCapacity = 1, kErrNonFinite = 2, kErrCellOverflow = 4, kErrBadInput = 8 };

// Effective pair coefficients of Eq. (6): E*, G*, beta(e), mu of a type pair.
struct PairCoef {
    double Es, Gs, beta, mu;
};

// One system of a batch.  Cells of system s occupy [c0, c0 + nc0*nc1*nc2).
struct SysDesc {
    double lo[3], hi[3], L[3], hL[3];
    double inv_w[3];        // cells per metre along each axis (nc / L)
    double g[3];
    double dt, hdt;
    double skin, disp_thr2; // rebuild when |disp|^2 > (skin/2)^2
    int64_t p0, p1;         // particle range
    int64_t c0;             // first global cell
    int32_t nc[3];
    int32_t periodic[3];
    int32_t wall;
    int32_t ntypes;
    int32_t coef0;          // first PairCoef of this system (ntypes x ntypes, row major)
    int32_t type0;          // first entry of this system in the per-type arrays
};

// Device flag block (one per context).
struct Flags {
    int32_t err;            // kErr* bits
    int32_t max_row;        // largest neighbour row seen at the last build
    int64_t abort_at;       // step number that needs a list rebuild (INT64_MAX = none)
    int64_t step_base;      // global number of the chunk's first step
    int64_t steps;          // completed steps
    int64_t builds;         // list builds
    unsigned long long contacts;  // sum over force evaluations of directed contacts
    unsigned long long wall_contacts;
    int64_t pad[8];
};

// Neighbour list (ELL, slot-major: slot k of particle i at k*n + i).
struct List {
    int32_t *nbr;    // [kmax][n] neighbour index (in the particle order of the build)
    int32_t *cnt;    // [n] row length
    double *xi;      // [3][kmax][n] tangential history of each slot
    uint64_t *mask;  // [n] bit k: slot k holds non-zero history; bit 63: wall history non-zero
    int32_t *ids;    // [n] particle ids in the order of the build
};

// ---------------------------------------------------------------- helpers

__host__ __device__ inline double min_image(double d, double L, double hL, int periodic) {
    if (periodic) {
        if (d > hL) d -= L;
        else if (d < -hL) d += L;
    }
    return d;
}

__host__ __device__ inline int cell_coord(double x, const SysDesc &s, int a) {
    double u = (x - s.lo[a]) * s.inv_w[a];
    int c;
    if (!(u >= 0.0)) c = 0;                          // also catches NaN
    else if (u >= (double)s.nc[a]) c = s.nc[a] - 1;
    else c = (int)u;
    return c;
}

// Contact of particle a with b (b_is_wall: flat wall z = 0, normal +z).
// Inputs are a's and b's state; xi is the slot's history (updated in place
// when update != 0).  Returns false (and touches nothing) when not in
// contact.  Outputs: force on a, tangential force and normal for the torque.
// The arithmetic order is fixed so that a pair evaluated from either side
// gives exactly opposite results (no contraction into fused multiply-adds
// anywhere in this library's force path).
struct ContactIn {
    double dx, dy, dz;   // x_a - x_b (minimum image); wall: (0, 0, z_a)
    double ra, rb;       // radii (wall: rb unused)
    double ma, mb;       // masses (wall: mb unused)
    double vrx, vry, vrz;        // v_a - v_b
    double wsx, wsy, wsz;        // r_a w_a + r_b w_b
};

__host__ __device__ inline bool contact_force(const ContactIn &c, bool wall, const PairCoef &k, double dt, bool update,
                                              double &xix, double &xiy, double &xiz, double &fx, double &fy, double &fz,
                                              double &ftx, double &fty, double &ftz, double &nx, double &ny,
                                              double &nz, double &fn_out) {
    double rs, dist;
    if (!wall) {
        double d2 = c.dx * c.dx + c.dy * c.dy + c.dz * c.dz;
        rs = c.ra + c.rb;
        if (!(d2 < rs * rs)) return false;
        dist = sqrt(d2);
    } else {
        rs = c.ra;
        if (!(c.dz < c.ra)) return false;
        dist = c.dz;
    }
    double delta = rs - dist;
    if (!(delta > 0.0)) return false;
    if (!wall) {
        nx = c.dx / dist; ny = c.dy / dist; nz = c.dz / dist;
    } else {
        nx = 0.0; ny = 0.0; nz = 1.0;
    }
    double R = wall ? c.ra : c.ra * c.rb / (c.ra + c.rb);
    double M = wall ? c.ma : c.ma * c.mb / (c.ma + c.mb);
    double sq = sqrt(R * delta);
    double kn = 4.0 / 3.0 * k.Es * sq;
    double kt = 8.0 * k.Gs * sq;
    double gn = -k.beta * sqrt(5.0 * M * kn);
    double gt = -k.beta * sqrt(10.0 / 3.0 * M * kt);
    double vn = c.vrx * nx + c.vry * ny + c.vrz * nz;
    double cx = c.wsy * nz - c.wsz * ny;
    double cy = c.wsz * nx - c.wsx * nz;
    double cz = c.wsx * ny - c.wsy * nx;
    double vtx = c.vrx - vn * nx - cx;
    double vty = c.vry - vn * ny - cy;
    double vtz = c.vrz - vn * nz - cz;
    double fn = kn * delta - gn * vn;
    double xn = xix * nx + xiy * ny + xiz * nz;
    double zx = xix - xn * nx, zy = xiy - xn * ny, zz = xiz - xn * nz;
    if (update) {
        zx = zx + vtx * dt;
        zy = zy + vty * dt;
        zz = zz + vtz * dt;
    }
    double tx = -kt * zx - gt * vtx;
    double ty = -kt * zy - gt * vty;
    double tz = -kt * zz - gt * vtz;
    double ft2 = tx * tx + ty * ty + tz * tz;
    double cap = k.mu * fabs(fn);
    if (ft2 > cap * cap) {
        double scale = cap / sqrt(ft2);
        tx = scale * tx; ty = scale * ty; tz = scale * tz;
        zx = -(tx + gt * vtx) / kt;
        zy = -(ty + gt * vty) / kt;
        zz = -(tz + gt * vtz) / kt;
    }
    if (update) { xix = zx; xiy = zy; xiz = zz; }
    fx = fn * nx + tx;
    fy = fn * ny + ty;
    fz = fn * nz + tz;
    ftx = tx; fty = ty; ftz = tz;
    fn_out = fn;
    return true;
}

}  // namespace dem
