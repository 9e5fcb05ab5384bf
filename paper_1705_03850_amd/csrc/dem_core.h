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
enum : int { kErrCapacity = 1, kErrNonFinite = 2, kErrCellOverflow = 4, kErrBadInput = 8, kErrStale = 16 };

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

// One system of a batch.  Cells of system s occupy [c0, c0 + nc0*nc1*nc2 + 1).
struct SysDesc {
    double lo[3], hi[3], L[3], hL[3];
    double inv_w[3];        // cells per metre along each axis (nc / L)
    double g[3];
    double dt, hdt;
    double skin, disp_thr2; // rebuild when |disp|^2 > (skin/2)^2
    double rmax;            // largest radius the system admits
    int64_t p0, p1;         // particle slots
    int64_t pe;             // end of the live particles, p0 <= pe <= p1 (slots after it are free)
    int64_t c0;             // first global cell; the system's cells, then one spare cell
                            // (index c0 + nc0 nc1 nc2) that the binning gives the free slots
    int32_t nc[3];
    int32_t periodic[3];
    int32_t wall;
    int32_t ntypes;
    int32_t coef0;          // first PairCoef of this system (ntypes x ntypes, row major)
    int32_t type0;          // first entry of this system in the per-type arrays
    int32_t stride;         // multi-rate stepping: one step of dt every `stride` substeps (else 1)
    int32_t nsurf;          // static wall surfaces of the system (Surf table entries surf0 ..)
    int32_t surf0;
    int32_t pad_s;
};

// Static wall surfaces around a vertical axis through (cx, cy): the inside of
// a cylinder (radius r0, z0 <= z <= z1), the inside of a cone frustum (radius
// r0 at z0, r1 at z1), a horizontal disk (radius r0 at height z0, touched from
// above) and a horizontal ring (radius r0 at z0, an edge).  The cone's unit
// generator (ur, uz), its length and its inward unit normal (mr, mz) in the
// meridional plane are derived on the host.
constexpr int kMaxSurf = 4;
enum : int { kSurfCylinder = 1, kSurfCone = 2, kSurfDisk = 3, kSurfRing = 4 };

struct Surf {
    int32_t kind, enabled;
    double cx, cy, z0, z1, r0, r1;
    double ur, uz, len, mr, mz;
    double mu;              // friction of a contact with the surface (< 0: the particle's own)
};

// A sphere of radius r at (x, y, z) touching surface w: the distance from the
// surface to the centre, 0 < dist < r, and the unit normal from the surface to
// the centre.  A centre on or behind the surface, beyond its extent (cylinder
// and cone: the normal's foot outside [z0, z1], disk: outside its radius) or
// on the axis has no contact with it.
__host__ __device__ inline bool surf_gap(const Surf &w, double x, double y, double z, double r, double &dist,
                                         double &nx, double &ny, double &nz) {
    const double dx = x - w.cx, dy = y - w.cy;
    const double rho = sqrt(dx * dx + dy * dy);
    if (w.kind == kSurfDisk) {
        const double h = z - w.z0;
        if (!(rho <= w.r0 && h > 0.0 && h < r)) return false;
        dist = h;
        nx = 0.0; ny = 0.0; nz = 1.0;
        return true;
    }
    if (!(rho > 0.0)) return false;
    const double ex = dx / rho, ey = dy / rho;
    if (w.kind == kSurfCylinder) {
        if (!(z >= w.z0 && z <= w.z1)) return false;
        const double g = w.r0 - rho;
        if (!(g > 0.0 && g < r)) return false;
        dist = g;
        nx = -ex; ny = -ey; nz = 0.0;
        return true;
    }
    if (w.kind == kSurfCone) {
        const double pr = rho - w.r0, pz = z - w.z0;
        const double t = pr * w.ur + pz * w.uz;   // along the generator from (r0, z0)
        if (!(t >= 0.0 && t <= w.len)) return false;
        const double g = pr * w.mr + pz * w.mz;   // towards the inside
        if (!(g > 0.0 && g < r)) return false;
        dist = g;
        nx = w.mr * ex; ny = w.mr * ey; nz = w.mz;
        return true;
    }
    if (w.kind == kSurfRing) {
        const double qr = rho - w.r0, qz = z - w.z0;
        const double d2 = qr * qr + qz * qz;
        if (!(d2 > 0.0 && d2 < r * r)) return false;
        const double d = sqrt(d2);
        dist = d;
        nx = qr / d * ex; ny = qr / d * ey; nz = qz / d;
        return true;
    }
    return false;
}

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
    int32_t reserved;
    int32_t pad0;
    int64_t call_base;      // multi-rate: step number before the first substep of the current dem_step
    int64_t step_end;       // multi-rate: step number of the call's last substep
    int64_t ex_removed;     // insertion event: spheres marked for removal
    int64_t ex_accepted;    //   candidates accepted
    int32_t ex_maxid;       //   largest live id of the context
    int32_t ex_err;         //   bad candidate, too many overlapping candidates, stale list
    int64_t pad[2];
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
    int32_t *nbr;    // [kmax][n] neighbour index (in the particle order of the build), slot
                     // major: slot q of particle i at q n + i, so that the slot-q reads of
                     // consecutive particles share lines
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

// A system's descriptor copied word by word into scalar registers (the value
// is the same for every lane).  Read through the table instead, its fields
// are loaded again after every store the compiler cannot tell apart from it:
// the slot loop of the fused step did that on every iteration.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ SysDesc uniform_sys(const SysDesc *p) {
    SysDesc s;
    const uint32_t *src = (const uint32_t *)p;
    uint32_t *dst = (uint32_t *)&s;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(SysDesc) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    return s;
}

// Periodic wrap of a drifted coordinate into [lo, hi).
__host__ __device__ inline double wrap_axis(double x, const SysDesc &s, int ax) {
    if (!s.periodic[ax]) return x;
    if (x >= s.hi[ax]) x -= s.L[ax];
    if (x < s.lo[ax]) x += s.L[ax];
    if (x >= s.hi[ax]) x = s.lo[ax];
    return x;
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

// The same with a wall of unit normal (nwx, nwy, nwz) (pointing from the wall
// to the particle's centre, at distance c.dz): a static surface seen as flat
// at the contact point.
__host__ __device__ inline bool contact_force_n(const ContactIn &c, bool wall, double nwx, double nwy, double nwz,
                                                const PairCoef &k, double dt, bool update, double &xix, double &xiy,
                                                double &xiz, double &fx, double &fy, double &fz, double &ftx,
                                                double &fty, double &ftz, double &nx, double &ny, double &nz,
                                                double &fn_out) {
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
        nx = nwx; ny = nwy; nz = nwz;
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

__host__ __device__ inline bool contact_force(const ContactIn &c, bool wall, const PairCoef &k, double dt, bool update,
                                              double &xix, double &xiy, double &xiz, double &fx, double &fy, double &fz,
                                              double &ftx, double &fty, double &ftz, double &nx, double &ny,
                                              double &nz, double &fn_out) {
    return contact_force_n(c, wall, 0.0, 0.0, 1.0, k, dt, update, xix, xiy, xiz, fx, fy, fz, ftx, fty, ftz, nx, ny, nz,
                           fn_out);
}

// Reverse mode of contact_force at the same inputs, for gradients of a
// trajectory with respect to the contact law.  Seeds: fb is the adjoint of the
// force on a, gb of g = n x F_t (both torques are -r g), zb of the updated
// history (used when update != 0).  Results: the adjoints of d = x_a - x_b
// (wall: of z_a in dbz), of v_a - v_b, of r_a w_a + r_b w_b, of the history
// before the update, and of the five folded coefficients.  Every branch
// (contact, Coulomb) is decided by the same expressions as in contact_force.
// With a's and b's roles swapped and the seeds mirrored (fb and zb negated,
// gb unchanged) every result flips sign exactly or stays the same, as the
// forward arithmetic does.  Returns false (and writes nothing) when not in
// contact.
struct ContactAdj {
    double dbx, dby, dbz;    // separation
    double vbx, vby, vbz;    // relative velocity
    double wbx, wby, wbz;    // r_a w_a + r_b w_b
    double xbx, xby, xbz;    // history before the update
    double kn0, kt0, gn0, gt0, mu;
};

__host__ __device__ inline bool contact_vjp(const ContactIn &c, bool wall, const PairCoef &k, double dt, bool update,
                                            double xix, double xiy, double xiz, double fbx, double fby, double fbz,
                                            double gbx, double gby, double gbz, double zbx, double zby, double zbz,
                                            ContactAdj &o) {
    // ---- forward values (the expressions of contact_force)
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
    const double delta = rs - dist;
    if (!(delta > 0.0)) return false;
    double nx, ny, nz, R, M, inv_d = 0.0;
    if (!wall) {
        inv_d = 1.0 / dist;
        nx = c.dx * inv_d; ny = c.dy * inv_d; nz = c.dz * inv_d;
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
    const double tx = -kt * zx - gt * vtx;
    const double ty = -kt * zy - gt * vty;
    const double tz = -kt * zz - gt * vtz;
    const double ft2 = tx * tx + ty * ty + tz * tz;
    const double cap = k.mu * fabs(fn);
    const bool slip = ft2 > cap * cap;
    double tpx = tx, tpy = ty, tpz = tz;   // total tangential force
    double s = 1.0, q = 0.0, inv_kt = 0.0, zpx = zx, zpy = zy, zpz = zz;
    if (slip) {
        q = sqrt(ft2);
        s = cap / q;
        tpx = s * tx; tpy = s * ty; tpz = s * tz;
        inv_kt = 1.0 / kt;
        zpx = -(tpx + gt * vtx) * inv_kt;
        zpy = -(tpy + gt * vty) * inv_kt;
        zpz = -(tpz + gt * vtz) * inv_kt;
    }
    if (!update) { zbx = 0.0; zby = 0.0; zbz = 0.0; }
    // ---- reverse sweep
    // f = f_n n + t',  g = n x t'
    double tbx = fbx + (gby * nz - gbz * ny);
    double tby = fby + (gbz * nx - gbx * nz);
    double tbz = fbz + (gbx * ny - gby * nx);
    double nbx = fn * fbx + (tpy * gbz - tpz * gby);
    double nby = fn * fby + (tpz * gbx - tpx * gbz);
    double nbz = fn * fbz + (tpx * gby - tpy * gbx);
    double fnb = fbx * nx + fby * ny + fbz * nz;
    double ktb = 0.0, gtb = 0.0, mub = 0.0, vtbx = 0.0, vtby = 0.0, vtbz = 0.0;
    double zqx, zqy, zqz;   // adjoint of the trial history z
    if (slip) {
        // z' = -(t' + g_t v_t) / k_t
        tbx = tbx + -inv_kt * zbx;
        tby = tby + -inv_kt * zby;
        tbz = tbz + -inv_kt * zbz;
        gtb = -inv_kt * (zbx * vtx + zby * vty + zbz * vtz);
        const double gk = gt * inv_kt;
        vtbx = -gk * zbx; vtby = -gk * zby; vtbz = -gk * zbz;
        ktb = -inv_kt * (zbx * zpx + zby * zpy + zbz * zpz);
        // t' = (cap / |t|) t
        const double tt = tx * tbx + ty * tby + tz * tbz;
        const double rr = tt / ft2;
        tbx = s * (tbx - tx * rr);
        tby = s * (tby - ty * rr);
        tbz = s * (tbz - tz * rr);
        const double capb = tt / q;
        mub = fabs(fn) * capb;
        fnb = fnb + (fn < 0.0 ? -k.mu * capb : k.mu * capb);
        zqx = 0.0; zqy = 0.0; zqz = 0.0;
    } else {
        zqx = zbx; zqy = zby; zqz = zbz;
    }
    // t = -k_t z - g_t v_t
    zqx = zqx + -kt * tbx;
    zqy = zqy + -kt * tby;
    zqz = zqz + -kt * tbz;
    ktb = ktb + -(zx * tbx + zy * tby + zz * tbz);
    gtb = gtb + -(vtx * tbx + vty * tby + vtz * tbz);
    vtbx = vtbx + -gt * tbx;
    vtby = vtby + -gt * tby;
    vtbz = vtbz + -gt * tbz;
    // z = (xi - (xi.n) n) + v_t dt
    if (update) {
        vtbx = vtbx + dt * zqx;
        vtby = vtby + dt * zqy;
        vtbz = vtbz + dt * zqz;
    }
    const double xnb = -(nx * zqx + ny * zqy + nz * zqz);
    nbx = nbx + -xn * zqx + xnb * xix;
    nby = nby + -xn * zqy + xnb * xiy;
    nbz = nbz + -xn * zqz + xnb * xiz;
    o.xbx = zqx + xnb * nx;
    o.xby = zqy + xnb * ny;
    o.xbz = zqz + xnb * nz;
    // f_n = k_n delta - g_n v_n
    const double knb = delta * fnb;
    double deltab = kn * fnb;
    const double gnb = -vn * fnb;
    double vnb = -gn * fnb;
    // v_t = v_r - v_n n - w_s x n
    vnb = vnb + -(nx * vtbx + ny * vtby + nz * vtbz);
    nbx = nbx + -vn * vtbx;
    nby = nby + -vn * vtby;
    nbz = nbz + -vn * vtbz;
    const double cbx = -vtbx, cby = -vtby, cbz = -vtbz;
    o.wbx = ny * cbz - nz * cby;
    o.wby = nz * cbx - nx * cbz;
    o.wbz = nx * cby - ny * cbx;
    nbx = nbx + (cby * c.wsz - cbz * c.wsy);
    nby = nby + (cbz * c.wsx - cbx * c.wsz);
    nbz = nbz + (cbx * c.wsy - cby * c.wsx);
    // v_n = v_r . n
    o.vbx = vtbx + vnb * nx;
    o.vby = vtby + vnb * ny;
    o.vbz = vtbz + vnb * nz;
    nbx = nbx + vnb * c.vrx;
    nby = nby + vnb * c.vry;
    nbz = nbz + vnb * c.vrz;
    // g = g0 sqrt(m* sqrt(R delta)),  k = k0 sqrt(R delta)
    o.gn0 = sg * gnb;
    o.gt0 = sg * gtb;
    o.kn0 = sq * knb;
    o.kt0 = sq * ktb;
    o.mu = mub;
    const double sgb = k.gn0 * gnb + k.gt0 * gtb;
    const double sqb = k.kn0 * knb + k.kt0 * ktb + sgb * (0.5 * M / sg);
    deltab = deltab + sqb * (0.5 * R / sq);
    if (wall) {
        o.dbx = 0.0; o.dby = 0.0; o.dbz = -deltab;
    } else {
        // delta = r_a + r_b - |d|,  n = d / |d|
        const double nn = nx * nbx + ny * nby + nz * nbz;
        o.dbx = (nbx - nx * nn) * inv_d - deltab * nx;
        o.dby = (nby - ny * nn) * inv_d - deltab * ny;
        o.dbz = (nbz - nz * nn) * inv_d - deltab * nz;
    }
    return true;
}

}  // namespace dem
