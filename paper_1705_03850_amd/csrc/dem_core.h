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

// Coefficients of Eq. (6) for a type pair, folded so that a contact needs
// three square roots and two divisions:
//   k_n = kn0 sqrt(R delta),        kn0 = (4/3) E*
//   k_t = kt0 sqrt(R delta),        kt0 = 8 G*
//   g_n = gn0 sqrt(m* sqrt(R delta)), gn0 = -beta sqrt((20/3) E*)   [= -beta sqrt(5 m* k_n)]
//   g_t = gt0 sqrt(m* sqrt(R delta)), gt0 = -beta sqrt((80/3) G*)   [= -beta sqrt((10/3) m* k_t)]
struct PairCoef {
    double kn0, kt0, gn0, gt0, mu;
    double pad[3];
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
// Packed working state of the step loop (one 32-byte record per particle and
// field group, so that a neighbour's position and radius arrive in one
// request): pos = (x, y, z, r), vel = (vx, vy, vz, m), spin = (wx, wy, wz, type).
struct alignas(32) D4 {
    double x, y, z, w;
};
struct alignas(16) D2 {
    double a, b;
};

struct List {
    int32_t *nbr;    // [n][kmax] neighbour index (in the particle order of the build)
    int32_t *cnt;    // [n] row length
    D4 *xi;          // [n][kmax] tangential history of each slot (x, y, z, unused): one
                     // 32-byte record, so a contact reads and writes one line
    uint64_t *mask;  // [n] bit k: slot k holds non-zero history; bit 63: wall history non-zero
    int32_t *ids;    // [n] particle ids in the order of the build
};

// ---------------------------------------------------------------- helpers

// Nearest periodic image of a coordinate difference (branch-free selects;
// the same result as subtracting L above L/2 and adding it below -L/2).
__host__ __device__ inline double min_image(double d, double L, double hL, int periodic) {
    const double dm = d - L, dp = d + L;
    const double r = d > hL ? dm : (d < -hL ? dp : d);
    return periodic ? r : d;
}

__host__ __device__ inline int cell_coord(double x, const SysDesc &s, int a) {
    double u = (x - s.lo[a]) * s.inv_w[a];
    int c;
    if (!(u >= 0.0)) c = 0;                          // also catches NaN
    else if (u >= (double)s.nc[a]) c = s.nc[a] - 1;
    else c = (int)u;
    return c;
}

// Contact of particle a with b (wall: flat wall z = 0, normal +z).  Inputs
// are a's and b's state; xi is the slot's history (updated in place when
// update != 0).  Returns false (and touches nothing) when not in contact.
// Outputs: force on a, tangential force and normal (for the torque), f_n.
// Every expression is either symmetric in a and b or flips sign exactly with
// the roles swapped, and nothing is contracted into fused multiply-adds, so a
// pair evaluated from either side gives exactly opposite forces and history.
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
    double R, M;
    if (!wall) {
        const double inv_d = 1.0 / dist;
        nx = c.dx * inv_d; ny = c.dy * inv_d; nz = c.dz * inv_d;
        // R = r_a r_b / (r_a + r_b) and m* = m_a m_b / (m_a + m_b) with one division
        const double sm = c.ma + c.mb;
        const double inv = 1.0 / (rs * sm);
        R = c.ra * c.rb * sm * inv;
        M = c.ma * c.mb * rs * inv;
    } else {
        nx = 0.0; ny = 0.0; nz = 1.0;
        R = c.ra;
        M = c.ma;
    }
    const double sq = sqrt(R * delta);
    const double kn = k.kn0 * sq;
    const double kt = k.kt0 * sq;
    const double sg = sqrt(M * sq);
    const double gn = k.gn0 * sg;
    const double gt = k.gt0 * sg;
    const double vn = c.vrx * nx + c.vry * ny + c.vrz * nz;
    const double cx = c.wsy * nz - c.wsz * ny;
    const double cy = c.wsz * nx - c.wsx * nz;
    const double cz = c.wsx * ny - c.wsy * nx;
    const double vtx = c.vrx - vn * nx - cx;
    const double vty = c.vry - vn * ny - cy;
    const double vtz = c.vrz - vn * nz - cz;
    const double fn = kn * delta - gn * vn;
    const double xn = xix * nx + xiy * ny + xiz * nz;
    double zx = xix - xn * nx, zy = xiy - xn * ny, zz = xiz - xn * nz;
    if (update) {
        zx = zx + vtx * dt;
        zy = zy + vty * dt;
        zz = zz + vtz * dt;
    }
    double tx = -kt * zx - gt * vtx;
    double ty = -kt * zy - gt * vty;
    double tz = -kt * zz - gt * vtz;
    const double ft2 = tx * tx + ty * ty + tz * tz;
    const double cap = k.mu * fabs(fn);
    if (ft2 > cap * cap) {
        const double scale = cap / sqrt(ft2);
        tx = scale * tx; ty = scale * ty; tz = scale * tz;
        const double inv_kt = 1.0 / kt;
        zx = -(tx + gt * vtx) * inv_kt;
        zy = -(ty + gt * vty) * inv_kt;
        zz = -(tz + gt * vtz) * inv_kt;
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
