// Host build of the library's per-contact arithmetic (dem_core.h), so that a
// CPU test can check the reverse mode against central differences of the
// forward.  Test infrastructure only.
#include "../../paper_1705_03850_amd/csrc/dem_core.h"

using namespace dem;

namespace {
ContactIn unpack_in(const double *in) {
    ContactIn c;
    c.dx = in[0]; c.dy = in[1]; c.dz = in[2];
    c.ra = in[3]; c.rb = in[4]; c.ma = in[5]; c.mb = in[6];
    c.vrx = in[7]; c.vry = in[8]; c.vrz = in[9];
    c.wsx = in[10]; c.wsy = in[11]; c.wsz = in[12];
    return c;
}
PairCoef unpack_coef(const double *k) {
    PairCoef p = {};
    p.kn0 = k[0]; p.kt0 = k[1]; p.gn0 = k[2]; p.gt0 = k[3]; p.mu = k[4];
    return p;
}
}  // namespace

extern "C" {

// in: dx dy dz ra rb ma mb vrx vry vrz wsx wsy wsz; xi[3]; coef[5]
// out: f[3], g = n x F_t [3], xi_new[3], slip flag; returns contact
int host_contact_force(const double *in, const double *xi, int wall, const double *coef, double dt, int update,
                       double *out) {
    ContactIn c = unpack_in(in);
    PairCoef k = unpack_coef(coef);
    double hx = xi[0], hy = xi[1], hz = xi[2];
    double fx, fy, fz, tx, ty, tz, nx, ny, nz, fn;
    if (!contact_force(c, wall != 0, k, dt, update != 0, hx, hy, hz, fx, fy, fz, tx, ty, tz, nx, ny, nz, fn))
        return 0;
    out[0] = fx; out[1] = fy; out[2] = fz;
    out[3] = ny * tz - nz * ty; out[4] = nz * tx - nx * tz; out[5] = nx * ty - ny * tx;
    out[6] = hx; out[7] = hy; out[8] = hz;
    const double ft2 = tx * tx + ty * ty + tz * tz;
    const double cap = k.mu * fabs(fn);
    out[9] = ft2 >= cap * cap * (1.0 - 1e-12) ? 1.0 : 0.0;
    return 1;
}

// seeds: fb[3], gb[3], zb[3]; out: db[3] vb[3] wb[3] xb[3] kn0 kt0 gn0 gt0 mu
int host_contact_vjp(const double *in, const double *xi, int wall, const double *coef, double dt, int update,
                     const double *seeds, double *out) {
    ContactIn c = unpack_in(in);
    PairCoef k = unpack_coef(coef);
    ContactAdj o;
    if (!contact_vjp(c, wall != 0, k, dt, update != 0, xi[0], xi[1], xi[2], seeds[0], seeds[1], seeds[2], seeds[3],
                     seeds[4], seeds[5], seeds[6], seeds[7], seeds[8], o))
        return 0;
    const double v[17] = {o.dbx, o.dby, o.dbz, o.vbx, o.vby, o.vbz, o.wbx, o.wby, o.wbz,
                          o.xbx, o.xby, o.xbz, o.kn0, o.kt0, o.gn0, o.gt0, o.mu};
    for (int i = 0; i < 17; ++i) out[i] = v[i];
    return 1;
}

}  // extern "C"
