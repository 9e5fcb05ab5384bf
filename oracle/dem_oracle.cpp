/*
 * dem_oracle.cpp -- plain, slow FP64 CPU reference of one soft-sphere DEM
 * contact step.  TEST INFRASTRUCTURE ONLY: the GPU library never links,
 * loads or calls this code, and this code shares nothing with it.
 *
 * What it computes (Queteschiner et al., "Adaptive Coarse-Graining for
 * Large-Scale DEM Simulations", CFD2017; cited by section and equation):
 *
 *   Newton's equations for translation and rotation          Sec. 2.1, Eq. (1)-(2)
 *   total force = gravity + sum of binary contact forces     Sec. 2.1, text after Eq. (2)
 *   normal spring-dashpot  f_n = k_n d_n - g_n d(d_n)/dt     Sec. 2.1, Eq. (3)
 *   tangential spring-dashpot with overlap history            Sec. 2.1, Eq. (4)
 *   truncation of the tangential overlap, f_t <= mu f_n       Sec. 2.1, Eq. (5)
 *   damped Hertz coefficients k_n, g_n, k_t, g_t, beta(e)     Sec. 2.1, Eq. (6)
 *   coarse-grain rule: E, nu, rho, e, mu fixed, r scaled      Sec. 2.2 (no explicit
 *       alpha appears: k ~ alpha and g ~ alpha^2 follow from the scaled radius)
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes of the repository):
 *   - effective properties are the Hertz-Mindlin harmonic combinations
 *       1/R = 1/r_i + 1/r_j, 1/m = 1/m_i + 1/m_j,
 *       1/E* = (1-nu_i^2)/E_i + (1-nu_j^2)/E_j,
 *       1/G* = 2(2-nu_i)(1+nu_i)/E_i + 2(2-nu_j)(1+nu_j)/E_j;
 *     the flat wall has the contacting particle's material and R, m of the particle;
 *     a pair of two types uses e = (e_i+e_j)/2 and mu = (mu_i+mu_j)/2;
 *   - n points from j to i; F_n = (k_n delta - g_n v_n) n, not clamped at zero;
 *     contact while d^2 < (r_i+r_j)^2 (strict);
 *   - the tangential history xi starts at zero, is reset when the pair is out of
 *     contact, is projected onto the current tangent plane (no rescaling) and then
 *     incremented by v_t dt; F_t* = -k_t xi - g_t v_t;
 *   - Coulomb: if |F_t*|^2 > (mu |f_n|)^2 the total tangential force is scaled to
 *     mu |f_n| and xi is solved back so that -k_t xi - g_t v_t equals it;
 *   - the contact lever arm is the radius r (v_t and the torque);
 *   - solid spheres, m = (4/3) pi rho r^3, I = (2/5) m r^2;
 *   - velocity Verlet (kick 1/2, drift, force, kick 1/2), forces evaluated with
 *     half-step velocities; a force evaluation may leave the history untouched
 *     (used once at the start of a run);
 *   - periodic images by minimum image; positions wrapped into [lo, hi).
 *
 * Every particle's force is accumulated gravity first, then its pair terms in
 * ascending partner id, then the wall, then an optional external force (the
 * correcting forces of the multi-level coupling, Sec. 2.3).  Pairs are visited
 * once (lower id first); the lower id's side holds the history.
 *
 * The scalar type is a template parameter so the same code also runs with
 * forward-mode dual numbers (derivatives with respect to per-type E, e, mu).
 *
 * Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -fPIC -shared dem_oracle.cpp -o liboracle.so
 */
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <chrono>
#include <map>
#include <omp.h>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

constexpr int NDIR = 6;  // tangent directions: E_0, E_1, e_0, e_1, mu_0, mu_1

/* ---------------------------------------------------------------- scalars */

struct Dual {
    double v;
    double d[NDIR];
    Dual() : v(0.0) { for (double &q : d) q = 0.0; }
    Dual(double x) : v(x) { for (double &q : d) q = 0.0; }  // NOLINT(implicit)
};
inline double val(double x) { return x; }
inline double val(const Dual &x) { return x.v; }
inline Dual operator+(const Dual &a, const Dual &b) { Dual c(a.v + b.v); for (int k = 0; k < NDIR; ++k) c.d[k] = a.d[k] + b.d[k]; return c; }
inline Dual operator-(const Dual &a, const Dual &b) { Dual c(a.v - b.v); for (int k = 0; k < NDIR; ++k) c.d[k] = a.d[k] - b.d[k]; return c; }
inline Dual operator-(const Dual &a) { Dual c(-a.v); for (int k = 0; k < NDIR; ++k) c.d[k] = -a.d[k]; return c; }
inline Dual operator*(const Dual &a, const Dual &b) { Dual c(a.v * b.v); for (int k = 0; k < NDIR; ++k) c.d[k] = a.d[k] * b.v + a.v * b.d[k]; return c; }
inline Dual operator/(const Dual &a, const Dual &b) {
    Dual c(a.v / b.v);
    for (int k = 0; k < NDIR; ++k) c.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return c;
}
inline Dual operator+(const Dual &a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual &b) { return Dual(a) + b; }
inline Dual operator-(const Dual &a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual &b) { return Dual(a) - b; }
inline Dual operator*(const Dual &a, double b) { Dual c(a.v * b); for (int k = 0; k < NDIR; ++k) c.d[k] = a.d[k] * b; return c; }
inline Dual operator*(double a, const Dual &b) { return b * a; }
inline Dual operator/(const Dual &a, double b) { return a / Dual(b); }
inline Dual operator/(double a, const Dual &b) { return Dual(a) / b; }
inline Dual &operator+=(Dual &a, const Dual &b) { a = a + b; return a; }
inline Dual &operator-=(Dual &a, const Dual &b) { a = a - b; return a; }
inline Dual sqrt(const Dual &a) {
    double s = std::sqrt(a.v);
    Dual c(s);
    for (int k = 0; k < NDIR; ++k) c.d[k] = a.d[k] / (2.0 * s);
    return c;
}
inline Dual log(const Dual &a) { Dual c(std::log(a.v)); for (int k = 0; k < NDIR; ++k) c.d[k] = a.d[k] / a.v; return c; }
inline Dual fabs(const Dual &a) { return a.v < 0.0 ? -a : a; }
using std::sqrt;
using std::log;
using std::fabs;

template <class S> struct V3 { S x, y, z; };

/* ------------------------------------------------------------ parameters */

struct Config {
    int ntypes;
    double E[4], nu[4], rho[4], e[4], mu[4];
    double dt, g[3], lo[3], hi[3];
    int periodic[3], wall_z0;
};

template <class S> struct PairCoef { S Es, Gs, beta, mu; };

template <class S> struct Particle {
    int id, type;
    double r, m, I, inv_m, inv_I;
    V3<S> x, v, w, f, t;
};

template <class S> struct PairRecord { int lo, hi; double fn_mag, f_mag, ft_mag, fncap, ft_normal; };

/* A static wall surface around the vertical axis through (cx, cy) (the silo
 * of Sec. 3): 1 the inside of a cylinder of radius r0 for z0 <= z <= z1, 2 the
 * inside of a cone frustum of radius r0 at z0 and r1 at z1, 3 a horizontal
 * disk of radius r0 at height z0 touched from above, 4 a horizontal ring
 * (circle) of radius r0 at z0.  A disabled surface is ignored. */
struct Surface {
    int kind, enabled;
    double cx, cy, z0, z1, r0, r1;
    double mu;   /* friction of a contact with it; < 0: the particle's own */
};

template <class S> struct Sim {
    Config cfg;
    S E[4], e[4], mu[4];  // material parameters as scalars (seeded for tangents)
    std::vector<Particle<S>> p;
    std::unordered_map<int, int> idx;                        // id -> index
    std::map<std::pair<int, int>, V3<S>> hist;               // (id_lo, id_hi) -> xi seen from id_lo
    std::map<int, V3<S>> whist;                              // id -> wall xi
    std::vector<PairRecord<S>> records;                      // last force evaluation
    std::vector<V3<double>> fext;                            // external force per particle (empty: none)
    std::vector<Surface> surf;                               // static wall surfaces
    std::map<std::pair<int, int>, V3<S>> shist;              // (id, surface) -> xi
    double rmax = 0.0;
};

/* Effective pair coefficients, Eq. (6) with the harmonic combinations above. */
template <class S> PairCoef<S> coef(const Sim<S> &s, int ti, int tj) {
    const Config &c = s.cfg;
    S inv_E = (1.0 - c.nu[ti] * c.nu[ti]) / s.E[ti] + (1.0 - c.nu[tj] * c.nu[tj]) / s.E[tj];
    S inv_G = 2.0 * (2.0 - c.nu[ti]) * (1.0 + c.nu[ti]) / s.E[ti] + 2.0 * (2.0 - c.nu[tj]) * (1.0 + c.nu[tj]) / s.E[tj];
    S e = (s.e[ti] + s.e[tj]) / 2.0;
    S mu = (s.mu[ti] + s.mu[tj]) / 2.0;
    S le = log(e);
    PairCoef<S> k;
    k.Es = 1.0 / inv_E;
    k.Gs = 1.0 / inv_G;
    k.beta = le / sqrt(le * le + M_PI * M_PI);
    k.mu = mu;
    return k;
}

inline double min_image(double d, double L, int periodic) {
    if (!periodic) return d;
    double hL = 0.5 * L;
    if (d > hL) d -= L;
    else if (d < -hL) d += L;
    return d;
}
template <class S> S min_image_s(const S &d, double L, int periodic) {
    if (!periodic) return d;
    double hL = 0.5 * L;
    if (val(d) > hL) return d - L;
    if (val(d) < -hL) return d + L;
    return d;
}

/*
 * One contact between particle a ("self") and b.  Computes the force on a
 * (f_out) and the tangential force ft (for the torques), updating xi in place
 * when update is set.  Wall: b == nullptr, normal +z, R = r_a, m* = m_a.
 * Returns false when not in contact.
 */
template <class S>
bool contact(const Sim<S> &s, const Particle<S> &a, const Particle<S> *b, V3<S> &xi, bool update, V3<S> &f_out,
             V3<S> &ft_out, V3<S> &n_out, PairRecord<S> *rec, const V3<double> *wn = nullptr, double wdist = 0.0,
             double wmu = -1.0) {
    const Config &c = s.cfg;
    V3<S> d;
    S dist;
    double rs;
    if (b) {
        d.x = min_image_s(a.x.x - b->x.x, c.hi[0] - c.lo[0], c.periodic[0]);
        d.y = min_image_s(a.x.y - b->x.y, c.hi[1] - c.lo[1], c.periodic[1]);
        d.z = min_image_s(a.x.z - b->x.z, c.hi[2] - c.lo[2], c.periodic[2]);
        S d2 = d.x * d.x + d.y * d.y + d.z * d.z;
        rs = a.r + b->r;
        if (!(val(d2) < rs * rs)) return false;
        dist = sqrt(d2);
    } else if (wn) {
        /* a static surface at distance wdist along its normal wn */
        rs = a.r;
        if (!(wdist < a.r)) return false;
        d.x = 0.0; d.y = 0.0; d.z = wdist;
        dist = wdist;
    } else {
        rs = a.r;
        if (!(val(a.x.z) < a.r)) return false;
        d.x = 0.0; d.y = 0.0; d.z = a.x.z;
        dist = a.x.z;
    }
    S delta = rs - dist;
    if (!(val(delta) > 0.0)) return false;
    V3<S> n;
    if (b) {
        n.x = d.x / dist; n.y = d.y / dist; n.z = d.z / dist;
    } else if (wn) {
        n.x = wn->x; n.y = wn->y; n.z = wn->z;
    } else {
        n.x = 0.0; n.y = 0.0; n.z = 1.0;
    }
    /* effective radius and mass */
    double R = b ? a.r * b->r / (a.r + b->r) : a.r;
    double M = b ? a.m * b->m / (a.m + b->m) : a.m;
    PairCoef<S> k = coef(s, a.type, b ? b->type : a.type);
    if (!b && wn && wmu >= 0.0) k.mu = wmu;   /* a surface with its own friction */
    /* Eq. (6) */
    S sq = sqrt(R * delta);
    S kn = 4.0 / 3.0 * k.Es * sq;
    S kt = 8.0 * k.Gs * sq;
    S gn = -k.beta * sqrt(5.0 * M * kn);
    S gt = -k.beta * sqrt(10.0 / 3.0 * M * kt);
    /* relative velocity of the contact point (lever arm r) */
    V3<S> vr = b ? V3<S>{a.v.x - b->v.x, a.v.y - b->v.y, a.v.z - b->v.z} : a.v;
    S vn = vr.x * n.x + vr.y * n.y + vr.z * n.z;
    V3<S> ws;
    if (b) {
        ws = {a.r * a.w.x + b->r * b->w.x, a.r * a.w.y + b->r * b->w.y, a.r * a.w.z + b->r * b->w.z};
    } else {
        ws = {a.r * a.w.x, a.r * a.w.y, a.r * a.w.z};
    }
    V3<S> wxn = {ws.y * n.z - ws.z * n.y, ws.z * n.x - ws.x * n.z, ws.x * n.y - ws.y * n.x};
    V3<S> vt = {vr.x - vn * n.x - wxn.x, vr.y - vn * n.y - wxn.y, vr.z - vn * n.z - wxn.z};
    /* Eq. (3) */
    S fn = kn * delta - gn * vn;
    /* Eq. (4): history projected onto the tangent plane, then advanced */
    S xn = xi.x * n.x + xi.y * n.y + xi.z * n.z;
    V3<S> z = {xi.x - xn * n.x, xi.y - xn * n.y, xi.z - xn * n.z};
    if (update) {
        z.x = z.x + vt.x * c.dt;
        z.y = z.y + vt.y * c.dt;
        z.z = z.z + vt.z * c.dt;
    }
    V3<S> ft = {-kt * z.x - gt * vt.x, -kt * z.y - gt * vt.y, -kt * z.z - gt * vt.z};
    /* Eq. (5): Coulomb truncation of the total tangential force */
    S ft2 = ft.x * ft.x + ft.y * ft.y + ft.z * ft.z;
    S cap = k.mu * fabs(fn);
    if (val(ft2) > val(cap * cap)) {
        S scale = cap / sqrt(ft2);
        ft = {scale * ft.x, scale * ft.y, scale * ft.z};
        z = {-(ft.x + gt * vt.x) / kt, -(ft.y + gt * vt.y) / kt, -(ft.z + gt * vt.z) / kt};
    }
    if (update) xi = z;
    f_out = {fn * n.x + ft.x, fn * n.y + ft.y, fn * n.z + ft.z};
    ft_out = ft;
    n_out = n;
    if (rec) {
        double fx = val(f_out.x), fy = val(f_out.y), fz = val(f_out.z);
        rec->fn_mag = std::fabs(val(fn));
        rec->f_mag = std::sqrt(fx * fx + fy * fy + fz * fz);
        rec->ft_mag = std::sqrt(val(ft.x) * val(ft.x) + val(ft.y) * val(ft.y) + val(ft.z) * val(ft.z));
        rec->fncap = val(cap);
        /* normal component of the tangential force (zero for a force in the tangent plane) */
        rec->ft_normal = std::fabs(val(ft.x) * val(n.x) + val(ft.y) * val(n.y) + val(ft.z) * val(n.z));
    }
    return true;
}

/* Candidate pairs (i < j by id) within d^2 < (r_i + r_j + extra)^2, visiting a
 * uniform grid of cells no smaller than the largest cut-off. */
template <class S> void grid_pairs(const Sim<S> &s, double extra, std::vector<std::pair<int, int>> &out) {
    const Config &c = s.cfg;
    double h = 2.0 * s.rmax + extra;
    int nc[3];
    for (int d = 0; d < 3; ++d) {
        double L = c.hi[d] - c.lo[d];
        nc[d] = std::max(1, (int)std::floor(L / h));
    }
    auto cell_of = [&](const Particle<S> &q, int ci[3]) {
        double xs[3] = {val(q.x.x), val(q.x.y), val(q.x.z)};
        for (int d = 0; d < 3; ++d) {
            double L = c.hi[d] - c.lo[d];
            int k = (int)std::floor((xs[d] - c.lo[d]) / L * nc[d]);
            if (c.periodic[d]) k = ((k % nc[d]) + nc[d]) % nc[d];
            else k = std::min(std::max(k, 0), nc[d] - 1);
            ci[d] = k;
        }
    };
    std::unordered_map<long long, std::vector<int>> cells;
    std::vector<std::array<int, 3>> pc(s.p.size());
    for (size_t i = 0; i < s.p.size(); ++i) {
        int ci[3];
        cell_of(s.p[i], ci);
        pc[i] = {ci[0], ci[1], ci[2]};
        cells[((long long)ci[2] * nc[1] + ci[1]) * nc[0] + ci[0]].push_back((int)i);
    }
    std::vector<int> order(s.p.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return s.p[a].id < s.p[b].id; });
    std::vector<int> cand;
    for (int i : order) {
        cand.clear();
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int cc[3] = {pc[i][0] + dx, pc[i][1] + dy, pc[i][2] + dz};
                    bool skip = false;
                    for (int d = 0; d < 3; ++d) {
                        if (c.periodic[d]) cc[d] = ((cc[d] % nc[d]) + nc[d]) % nc[d];
                        else if (cc[d] < 0 || cc[d] >= nc[d]) skip = true;
                    }
                    if (skip) continue;
                    auto it = cells.find(((long long)cc[2] * nc[1] + cc[1]) * nc[0] + cc[0]);
                    if (it == cells.end()) continue;
                    for (int j : it->second)
                        if (s.p[j].id > s.p[i].id) cand.push_back(j);
                }
        std::sort(cand.begin(), cand.end(), [&](int a, int b) { return s.p[a].id < s.p[b].id; });
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        for (int j : cand) {
            double dx = min_image(val(s.p[i].x.x) - val(s.p[j].x.x), c.hi[0] - c.lo[0], c.periodic[0]);
            double dy = min_image(val(s.p[i].x.y) - val(s.p[j].x.y), c.hi[1] - c.lo[1], c.periodic[1]);
            double dz = min_image(val(s.p[i].x.z) - val(s.p[j].x.z), c.hi[2] - c.lo[2], c.periodic[2]);
            double d2 = dx * dx + dy * dy + dz * dz;
            double cut = s.p[i].r + s.p[j].r + extra;
            if (d2 < cut * cut) out.push_back({i, j});
        }
    }
}

/* The same set by checking every pair: O(N^2), the definition itself. */
template <class S> void brute_pairs(const Sim<S> &s, double extra, std::vector<std::pair<int, int>> &out) {
    const Config &c = s.cfg;
    for (size_t i = 0; i < s.p.size(); ++i)
        for (size_t j = 0; j < s.p.size(); ++j) {
            if (s.p[j].id <= s.p[i].id) continue;
            double dx = min_image(val(s.p[i].x.x) - val(s.p[j].x.x), c.hi[0] - c.lo[0], c.periodic[0]);
            double dy = min_image(val(s.p[i].x.y) - val(s.p[j].x.y), c.hi[1] - c.lo[1], c.periodic[1]);
            double dz = min_image(val(s.p[i].x.z) - val(s.p[j].x.z), c.hi[2] - c.lo[2], c.periodic[2]);
            double d2 = dx * dx + dy * dy + dz * dz;
            double cut = s.p[i].r + s.p[j].r + extra;
            if (d2 < cut * cut) out.push_back({(int)i, (int)j});
        }
    std::sort(out.begin(), out.end(), [&](const std::pair<int, int> &a, const std::pair<int, int> &b) {
        if (s.p[a.first].id != s.p[b.first].id) return s.p[a.first].id < s.p[b.first].id;
        return s.p[a.second].id < s.p[b.second].id;
    });
}

/* Contact of a sphere (centre (x, y, z), radius r) with surface w, from the
 * definitions: the nearest point of the surface piece to the centre, the
 * distance d to it and the unit vector n from it to the centre; in contact
 * when the centre is on the inner side and 0 < d < r.  Cylinder and cone are
 * handled in the meridional half-plane through the centre (distance rho from
 * the axis, height z), where they are a vertical segment and a slanted one;
 * a centre whose perpendicular foot lies off the segment has no contact. */
static bool surface_contact(const Surface &w, double x, double y, double z, double r, double &dist, V3<double> &n) {
    if (!w.enabled) return false;
    const double dx = x - w.cx, dy = y - w.cy;
    const double rho = std::sqrt(dx * dx + dy * dy);
    if (w.kind == 3) {                                   /* disk, from above */
        if (rho > w.r0) return false;
        const double d = z - w.z0;
        if (!(d > 0.0 && d < r)) return false;
        dist = d;
        n = {0.0, 0.0, 1.0};
        return true;
    }
    if (rho == 0.0) return false;                        /* on the axis: no direction */
    if (w.kind == 1) {                                   /* cylinder, from inside */
        if (z < w.z0 || z > w.z1) return false;
        const double d = w.r0 - rho;
        if (!(d > 0.0 && d < r)) return false;
        dist = d;
        n = {-dx / rho, -dy / rho, 0.0};
        return true;
    }
    if (w.kind == 2) {                                   /* cone, from inside */
        const double sr = w.r1 - w.r0, sz = w.z1 - w.z0;
        const double t = ((rho - w.r0) * sr + (z - w.z0) * sz) / (sr * sr + sz * sz);
        if (t < 0.0 || t > 1.0) return false;
        const double qr = rho - (w.r0 + t * sr), qz = z - (w.z0 + t * sz);
        const double d = std::sqrt(qr * qr + qz * qz);
        const double side = sr * (z - w.z0) - sz * (rho - w.r0);   /* > 0: towards the axis */
        if (!(side > 0.0 && d > 0.0 && d < r)) return false;
        dist = d;
        n = {qr / d * (dx / rho), qr / d * (dy / rho), qz / d};
        return true;
    }
    if (w.kind == 4) {                                   /* ring */
        const double qr = rho - w.r0, qz = z - w.z0;
        const double d = std::sqrt(qr * qr + qz * qz);
        if (!(d > 0.0 && d < r)) return false;
        dist = d;
        n = {qr / d * (dx / rho), qr / d * (dy / rho), qz / d};
        return true;
    }
    return false;
}

/* Total force and torque on every particle (Sec. 2.1). */
template <class S> void forces(Sim<S> &s, bool update) {
    const Config &c = s.cfg;
    for (auto &q : s.p) {
        q.f = {q.m * c.g[0], q.m * c.g[1], q.m * c.g[2]};
        q.t = {0.0, 0.0, 0.0};
    }
    s.records.clear();
    std::vector<std::pair<int, int>> cand;
    grid_pairs(s, 0.0, cand);  // ordered by the lower id, then ascending partner id
    std::map<std::pair<int, int>, V3<S>> next;
    for (auto &pr : cand) {
        Particle<S> &a = s.p[pr.first];
        Particle<S> &b = s.p[pr.second];
        std::pair<int, int> key{a.id, b.id};
        auto it = s.hist.find(key);
        V3<S> xi = it == s.hist.end() ? V3<S>{0.0, 0.0, 0.0} : it->second;
        V3<S> f, ft, n;
        PairRecord<S> rec{a.id, b.id, 0, 0, 0, 0, 0};
        if (!contact(s, a, &b, xi, update, f, ft, n, &rec)) continue;
        s.records.push_back(rec);
        if (update) next[key] = xi;
        a.f = {a.f.x + f.x, a.f.y + f.y, a.f.z + f.z};
        b.f = {b.f.x - f.x, b.f.y - f.y, b.f.z - f.z};
        V3<S> nxf = {n.y * ft.z - n.z * ft.y, n.z * ft.x - n.x * ft.z, n.x * ft.y - n.y * ft.x};
        a.t = {a.t.x - a.r * nxf.x, a.t.y - a.r * nxf.y, a.t.z - a.r * nxf.z};
        b.t = {b.t.x - b.r * nxf.x, b.t.y - b.r * nxf.y, b.t.z - b.r * nxf.z};
    }
    if (update) s.hist.swap(next);
    if (c.wall_z0) {
        std::map<int, V3<S>> wnext;
        for (auto &a : s.p) {
            auto it = s.whist.find(a.id);
            V3<S> xi = it == s.whist.end() ? V3<S>{0.0, 0.0, 0.0} : it->second;
            V3<S> f, ft, n;
            PairRecord<S> rec{a.id, -1, 0, 0, 0, 0, 0};
            if (!contact(s, a, (const Particle<S> *)nullptr, xi, update, f, ft, n, &rec)) continue;
            s.records.push_back(rec);
            if (update) wnext[a.id] = xi;
            a.f = {a.f.x + f.x, a.f.y + f.y, a.f.z + f.z};
            V3<S> nxf = {n.y * ft.z - n.z * ft.y, n.z * ft.x - n.x * ft.z, n.x * ft.y - n.y * ft.x};
            a.t = {a.t.x - a.r * nxf.x, a.t.y - a.r * nxf.y, a.t.z - a.r * nxf.z};
        }
        if (update) s.whist.swap(wnext);
    }
    /* static surfaces, in their order (double precision runs only) */
    if (!s.surf.empty()) {
        std::map<std::pair<int, int>, V3<S>> snext;
        for (auto &a : s.p)
            for (size_t k = 0; k < s.surf.size(); ++k) {
                double dist;
                V3<double> wn;
                if (!surface_contact(s.surf[k], val(a.x.x), val(a.x.y), val(a.x.z), a.r, dist, wn)) continue;
                std::pair<int, int> key{a.id, (int)k};
                auto it = s.shist.find(key);
                V3<S> xi = it == s.shist.end() ? V3<S>{0.0, 0.0, 0.0} : it->second;
                V3<S> f, ft, n;
                PairRecord<S> rec{a.id, -2 - (int)k, 0, 0, 0, 0, 0};
                if (!contact(s, a, (const Particle<S> *)nullptr, xi, update, f, ft, n, &rec, &wn, dist,
                             s.surf[k].mu))
                    continue;
                s.records.push_back(rec);
                if (update) snext[key] = xi;
                a.f = {a.f.x + f.x, a.f.y + f.y, a.f.z + f.z};
                V3<S> nxf = {n.y * ft.z - n.z * ft.y, n.z * ft.x - n.x * ft.z, n.x * ft.y - n.y * ft.x};
                a.t = {a.t.x - a.r * nxf.x, a.t.y - a.r * nxf.y, a.t.z - a.r * nxf.z};
            }
        if (update) s.shist.swap(snext);
    }
    /* external forces (the coupling's correcting forces, Sec. 2.3), added last */
    if (!s.fext.empty())
        for (size_t i = 0; i < s.p.size(); ++i)
            s.p[i].f = {s.p[i].f.x + s.fext[i].x, s.p[i].f.y + s.fext[i].y, s.p[i].f.z + s.fext[i].z};
}

template <class S> S wrap(S x, double lo, double hi, int periodic) {
    if (!periodic) return x;
    double L = hi - lo;
    if (val(x) >= hi) x = x - L;
    if (val(x) < lo) x = x + L;
    if (val(x) >= hi) x = S(lo);
    return x;
}

/* Velocity Verlet for Eq. (1)-(2): kick 1/2, drift, forces, kick 1/2. */
template <class S> void kick(Sim<S> &s) {
    double h = 0.5 * s.cfg.dt;
    for (auto &q : s.p) {
        q.v = {q.v.x + h * (q.f.x * q.inv_m), q.v.y + h * (q.f.y * q.inv_m), q.v.z + h * (q.f.z * q.inv_m)};
        q.w = {q.w.x + h * (q.t.x * q.inv_I), q.w.y + h * (q.t.y * q.inv_I), q.w.z + h * (q.t.z * q.inv_I)};
    }
}
template <class S> void drift(Sim<S> &s) {
    const Config &c = s.cfg;
    for (auto &q : s.p) {
        q.x = {q.x.x + c.dt * q.v.x, q.x.y + c.dt * q.v.y, q.x.z + c.dt * q.v.z};
        q.x.x = wrap(q.x.x, c.lo[0], c.hi[0], c.periodic[0]);
        q.x.y = wrap(q.x.y, c.lo[1], c.hi[1], c.periodic[1]);
        q.x.z = wrap(q.x.z, c.lo[2], c.hi[2], c.periodic[2]);
    }
}
template <class S> void step(Sim<S> &s, int n) {
    for (int k = 0; k < n; ++k) {
        kick(s);
        drift(s);
        forces(s, true);
        kick(s);
    }
}

template <class S>
Sim<S> *make(const Config *cfg, int n, const double *x, const double *v, const double *w, const double *r,
             const int *type, const int *id) {
    Sim<S> *s = new Sim<S>();
    s->cfg = *cfg;
    for (int t = 0; t < cfg->ntypes; ++t) { s->E[t] = cfg->E[t]; s->e[t] = cfg->e[t]; s->mu[t] = cfg->mu[t]; }
    s->p.resize(n);
    for (int i = 0; i < n; ++i) {
        Particle<S> &q = s->p[i];
        q.id = id[i];
        q.type = type[i];
        q.r = r[i];
        q.m = 4.0 / 3.0 * M_PI * cfg->rho[q.type] * q.r * q.r * q.r;
        q.I = 0.4 * q.m * q.r * q.r;
        q.inv_m = 1.0 / q.m;
        q.inv_I = 1.0 / q.I;
        q.x = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        q.v = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        q.w = {w[3 * i], w[3 * i + 1], w[3 * i + 2]};
        q.f = {0.0, 0.0, 0.0};
        q.t = {0.0, 0.0, 0.0};
        s->idx[q.id] = i;
        s->rmax = std::max(s->rmax, q.r);
    }
    return s;
}

using SimD = Sim<double>;
using SimT = Sim<Dual>;

/* ------------------------------------------------------------------------
 * All-cores timing leg (OpenMP).  The same steps as step() above, with the
 * force evaluation written as a gather: every particle visits its own
 * partners in ascending id and computes each pair from its own side, which
 * gives exactly the negated force and history of the lower id's evaluation,
 * so the sums come out bit for bit as in forces() (a test checks this).  The
 * history lives in per-particle rows (partners of higher id, sorted by id)
 * during the call and goes back to the map at its end.  Used only to time the
 * oracle on all host cores; every parity check runs the serial path.
 * ---------------------------------------------------------------------- */
/* Rows of the own side of every pair: for particle i, the partners of higher
 * id in ascending id (index and history), at most kRow of them. */
constexpr int kRow = 48;
struct Rows {
    std::vector<int> cnt, j;
    std::vector<V3<double>> xi;
    void init(int n) { cnt.assign(n, 0); j.assign((size_t)n * kRow, 0); xi.assign((size_t)n * kRow, V3<double>{0, 0, 0}); }
};

static const V3<double> *row_find(const Rows &r, const SimD &s, int i, int j) {
    int lo = 0, hi = r.cnt[i];
    const int *rj = &r.j[(size_t)i * kRow];
    const int idj = s.p[j].id;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (s.p[rj[mid]].id < idj) lo = mid + 1;
        else hi = mid;
    }
    return lo < r.cnt[i] && rj[lo] == j ? &r.xi[(size_t)i * kRow + lo] : nullptr;
}

static void parallel_forces(SimD &s, Rows &rows, Rows &next, std::vector<V3<double>> &wxi, std::vector<char> &whas,
                            bool update) {
    const Config &c = s.cfg;
    const int n = (int)s.p.size();
    double h = 2.0 * s.rmax;
    int nc[3];
    for (int d = 0; d < 3; ++d) nc[d] = std::max(1, (int)std::floor((c.hi[d] - c.lo[d]) / h));
    std::vector<int> cell(n), start((size_t)nc[0] * nc[1] * nc[2] + 1, 0), order(n);
    auto coord = [&](double x, int d) {
        double L = c.hi[d] - c.lo[d];
        int k = (int)std::floor((x - c.lo[d]) / L * nc[d]);
        if (c.periodic[d]) k = ((k % nc[d]) + nc[d]) % nc[d];
        else k = std::min(std::max(k, 0), nc[d] - 1);
        return k;
    };
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        cell[i] = (coord(s.p[i].x.z, 2) * nc[1] + coord(s.p[i].x.y, 1)) * nc[0] + coord(s.p[i].x.x, 0);
    for (int i = 0; i < n; ++i) ++start[cell[i] + 1];
    for (size_t k = 1; k < start.size(); ++k) start[k] += start[k - 1];
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int i = 0; i < n; ++i) order[fill[cell[i]]++] = i;
    }
    bool overflow = false;
#pragma omp parallel
    {
        std::vector<int> cand;
#pragma omp for schedule(dynamic, 256)
        for (int i = 0; i < n; ++i) {
            Particle<double> &a = s.p[i];
            a.f = {a.m * c.g[0], a.m * c.g[1], a.m * c.g[2]};
            a.t = {0.0, 0.0, 0.0};
            const int ci[3] = {coord(a.x.x, 0), coord(a.x.y, 1), coord(a.x.z, 2)};
            cand.clear();
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int cc[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
                        bool skip = false;
                        for (int d = 0; d < 3; ++d) {
                            if (c.periodic[d]) cc[d] = ((cc[d] % nc[d]) + nc[d]) % nc[d];
                            else if (cc[d] < 0 || cc[d] >= nc[d]) skip = true;
                        }
                        if (skip) continue;
                        const int k = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
                        for (int q = start[k]; q < start[k + 1]; ++q)
                            if (order[q] != i) cand.push_back(order[q]);
                    }
            std::sort(cand.begin(), cand.end(), [&](int p, int q) { return s.p[p].id < s.p[q].id; });
            cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
            int own_n = 0;
            for (int j : cand) {
                const Particle<double> &b = s.p[j];
                const bool own = a.id < b.id;
                V3<double> x = {0.0, 0.0, 0.0};
                if (own) {
                    if (const V3<double> *p = row_find(rows, s, i, j)) x = *p;
                } else if (const V3<double> *p = row_find(rows, s, j, i)) {
                    x = {-p->x, -p->y, -p->z};
                }
                V3<double> f, ft, nn;
                if (!contact(s, a, &b, x, update, f, ft, nn, (PairRecord<double> *)nullptr)) continue;
                if (own && update) {
                    if (own_n < kRow) {
                        next.j[(size_t)i * kRow + own_n] = j;
                        next.xi[(size_t)i * kRow + own_n] = x;
                        ++own_n;
                    } else {
                        overflow = true;
                    }
                }
                a.f = {a.f.x + f.x, a.f.y + f.y, a.f.z + f.z};
                V3<double> nxf = {nn.y * ft.z - nn.z * ft.y, nn.z * ft.x - nn.x * ft.z, nn.x * ft.y - nn.y * ft.x};
                a.t = {a.t.x - a.r * nxf.x, a.t.y - a.r * nxf.y, a.t.z - a.r * nxf.z};
            }
            if (update) next.cnt[i] = own_n;
            if (c.wall_z0) {
                V3<double> x = whas[i] ? wxi[i] : V3<double>{0.0, 0.0, 0.0};
                V3<double> f, ft, nn;
                if (contact(s, a, (const Particle<double> *)nullptr, x, update, f, ft, nn,
                            (PairRecord<double> *)nullptr)) {
                    a.f = {a.f.x + f.x, a.f.y + f.y, a.f.z + f.z};
                    V3<double> nxf = {nn.y * ft.z - nn.z * ft.y, nn.z * ft.x - nn.x * ft.z, nn.x * ft.y - nn.y * ft.x};
                    a.t = {a.t.x - a.r * nxf.x, a.t.y - a.r * nxf.y, a.t.z - a.r * nxf.z};
                    if (update) { wxi[i] = x; whas[i] = 1; }
                } else if (update) {
                    whas[i] = 0;
                }
            }
            if (!s.fext.empty()) a.f = {a.f.x + s.fext[i].x, a.f.y + s.fext[i].y, a.f.z + s.fext[i].z};
        }
    }
    if (overflow) std::abort();   // more than kRow contacts of one sphere: not a packing of spheres
    if (update) std::swap(rows, next);
}

}  // namespace

extern "C" {

/* nsteps steps on all cores (the timing leg above); returns the threads used
 * and, in *seconds, the time of the step loop alone (steady clock).  The state
 * and histories afterwards are those of orc_step. */
int orc_step_parallel(void *h, int nsteps, double *seconds) {
    if (!((SimD *)h)->surf.empty()) return -1;   /* the gather form has no surfaces */
    SimD *s = (SimD *)h;
    const int n = (int)s->p.size();
    Rows rows, next;
    rows.init(n);
    next.init(n);
    for (auto &kv : s->hist) {
        int i = s->idx[kv.first.first], j = s->idx[kv.first.second];
        int &k = rows.cnt[i];
        if (k >= kRow) std::abort();
        rows.j[(size_t)i * kRow + k] = j;
        rows.xi[(size_t)i * kRow + k] = kv.second;
        ++k;
    }
    std::vector<V3<double>> wxi(n, V3<double>{0.0, 0.0, 0.0});
    std::vector<char> whas(n, 0);
    for (auto &kv : s->whist) {
        int i = s->idx[kv.first];
        wxi[i] = kv.second;
        whas[i] = 1;
    }
    const double hdt = 0.5 * s->cfg.dt;
    const auto t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < nsteps; ++k) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            Particle<double> &q = s->p[i];
            q.v = {q.v.x + hdt * (q.f.x * q.inv_m), q.v.y + hdt * (q.f.y * q.inv_m), q.v.z + hdt * (q.f.z * q.inv_m)};
            q.w = {q.w.x + hdt * (q.t.x * q.inv_I), q.w.y + hdt * (q.t.y * q.inv_I), q.w.z + hdt * (q.t.z * q.inv_I)};
            const Config &c = s->cfg;
            q.x = {q.x.x + c.dt * q.v.x, q.x.y + c.dt * q.v.y, q.x.z + c.dt * q.v.z};
            q.x.x = wrap(q.x.x, c.lo[0], c.hi[0], c.periodic[0]);
            q.x.y = wrap(q.x.y, c.lo[1], c.hi[1], c.periodic[1]);
            q.x.z = wrap(q.x.z, c.lo[2], c.hi[2], c.periodic[2]);
        }
        parallel_forces(*s, rows, next, wxi, whas, true);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            Particle<double> &q = s->p[i];
            q.v = {q.v.x + hdt * (q.f.x * q.inv_m), q.v.y + hdt * (q.f.y * q.inv_m), q.v.z + hdt * (q.f.z * q.inv_m)};
            q.w = {q.w.x + hdt * (q.t.x * q.inv_I), q.w.y + hdt * (q.t.y * q.inv_I), q.w.z + hdt * (q.t.z * q.inv_I)};
        }
    }
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    s->hist.clear();
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < rows.cnt[i]; ++k)
            s->hist[{s->p[i].id, s->p[rows.j[(size_t)i * kRow + k]].id}] = rows.xi[(size_t)i * kRow + k];
    s->whist.clear();
    for (int i = 0; i < n; ++i)
        if (whas[i]) s->whist[s->p[i].id] = wxi[i];
    s->records.clear();
    int threads = 1;
#pragma omp parallel
    {
#pragma omp single
        threads = omp_get_num_threads();
    }
    return threads;
}

}  // extern "C"

extern "C" {

typedef Config orc_config;

void *orc_new(const orc_config *cfg, int n, const double *x, const double *v, const double *w, const double *r,
              const int *type, const int *id) {
    return make<double>(cfg, n, x, v, w, r, type, id);
}

void orc_free(void *h) { delete (SimD *)h; }

int orc_n(void *h) { return (int)((SimD *)h)->p.size(); }

/* State in input order, (n, 3) row-major. Any pointer may be null. */
void orc_get(void *h, double *x, double *v, double *w, double *f, double *t) {
    SimD *s = (SimD *)h;
    for (size_t i = 0; i < s->p.size(); ++i) {
        const Particle<double> &q = s->p[i];
        if (x) { x[3 * i] = q.x.x; x[3 * i + 1] = q.x.y; x[3 * i + 2] = q.x.z; }
        if (v) { v[3 * i] = q.v.x; v[3 * i + 1] = q.v.y; v[3 * i + 2] = q.v.z; }
        if (w) { w[3 * i] = q.w.x; w[3 * i + 1] = q.w.y; w[3 * i + 2] = q.w.z; }
        if (f) { f[3 * i] = q.f.x; f[3 * i + 1] = q.f.y; f[3 * i + 2] = q.f.z; }
        if (t) { t[3 * i] = q.t.x; t[3 * i + 1] = q.t.y; t[3 * i + 2] = q.t.z; }
    }
}

void orc_set(void *h, const double *x, const double *v, const double *w, const double *f, const double *t) {
    SimD *s = (SimD *)h;
    for (size_t i = 0; i < s->p.size(); ++i) {
        Particle<double> &q = s->p[i];
        if (x) q.x = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        if (v) q.v = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        if (w) q.w = {w[3 * i], w[3 * i + 1], w[3 * i + 2]};
        if (f) q.f = {f[3 * i], f[3 * i + 1], f[3 * i + 2]};
        if (t) q.t = {t[3 * i], t[3 * i + 1], t[3 * i + 2]};
    }
}

/* Masses and inertias as the oracle computes them, input order. */
void orc_get_mass(void *h, double *m, double *I) {
    SimD *s = (SimD *)h;
    for (size_t i = 0; i < s->p.size(); ++i) { m[i] = s->p[i].m; I[i] = s->p[i].I; }
}

void orc_forces(void *h, int update_history) { forces(*(SimD *)h, update_history != 0); }

void orc_step(void *h, int nsteps) { step(*(SimD *)h, nsteps); }

void orc_kick(void *h) { kick(*(SimD *)h); }
void orc_drift(void *h) { drift(*(SimD *)h); }

/* Pair history, (id_lo, id_hi) ascending; xi is seen from id_lo. */
long orc_history(void *h, int *lo, int *hi, double *xi, long cap) {
    SimD *s = (SimD *)h;
    long k = 0;
    for (auto &kv : s->hist) {
        if (k < cap) {
            lo[k] = kv.first.first; hi[k] = kv.first.second;
            xi[3 * k] = kv.second.x; xi[3 * k + 1] = kv.second.y; xi[3 * k + 2] = kv.second.z;
        }
        ++k;
    }
    return k;
}

void orc_set_history(void *h, long count, const int *lo, const int *hi, const double *xi) {
    SimD *s = (SimD *)h;
    s->hist.clear();
    for (long k = 0; k < count; ++k) {
        int a = lo[k], b = hi[k];
        V3<double> z = {xi[3 * k], xi[3 * k + 1], xi[3 * k + 2]};
        if (a > b) { std::swap(a, b); z = {-z.x, -z.y, -z.z}; }
        s->hist[{a, b}] = z;
    }
}

long orc_wall_history(void *h, int *id, double *xi, long cap) {
    SimD *s = (SimD *)h;
    long k = 0;
    for (auto &kv : s->whist) {
        if (k < cap) {
            id[k] = kv.first;
            xi[3 * k] = kv.second.x; xi[3 * k + 1] = kv.second.y; xi[3 * k + 2] = kv.second.z;
        }
        ++k;
    }
    return k;
}

void orc_set_wall_history(void *h, long count, const int *id, const double *xi) {
    SimD *s = (SimD *)h;
    s->whist.clear();
    for (long k = 0; k < count; ++k) s->whist[id[k]] = {xi[3 * k], xi[3 * k + 1], xi[3 * k + 2]};
}

/* Unordered pairs (id_lo < id_hi), ascending, with d^2 < (r_i + r_j + extra)^2.
 * brute != 0 checks all N^2 pairs; otherwise a uniform cell grid is used. */
long orc_pairs(void *h, double extra, int brute, int *lo, int *hi, long cap) {
    SimD *s = (SimD *)h;
    std::vector<std::pair<int, int>> out;
    if (brute) brute_pairs(*s, extra, out);
    else grid_pairs(*s, extra, out);
    long k = 0;
    for (auto &pr : out) {
        if (k < cap) { lo[k] = s->p[pr.first].id; hi[k] = s->p[pr.second].id; }
        ++k;
    }
    return k;
}

/* Per-contact records of the last force evaluation: ids (hi = -1 for the
 * wall) and magnitudes |f_n| (scalar normal force), |F_ij|, |F_t|, the
 * Coulomb cap mu |f_n| and |F_t . n| (ftn may be null). */
long orc_records(void *h, int *lo, int *hi, double *fn, double *fmag, double *ftmag, double *cap, double *ftn,
                 long capn) {
    SimD *s = (SimD *)h;
    long k = 0;
    for (auto &r : s->records) {
        if (k < capn) {
            lo[k] = r.lo; hi[k] = r.hi; fn[k] = r.fn_mag; fmag[k] = r.f_mag; ftmag[k] = r.ft_mag; cap[k] = r.fncap;
            if (ftn) ftn[k] = r.ft_normal;
        }
        ++k;
    }
    return k;
}

/* Static wall surfaces: count records of 9 doubles (kind, enabled, cx, cy, z0,
 * z1, r0, r1, mu).  The history of a surface whose record changed is dropped. */
void orc_set_surfaces(void *h, int count, const double *desc) {
    SimD *s = (SimD *)h;
    std::vector<Surface> next(count);
    for (int k = 0; k < count; ++k) {
        const double *q = desc + 9 * k;
        next[k] = {(int)q[0], (int)q[1], q[2], q[3], q[4], q[5], q[6], q[7], q[8]};
    }
    std::map<std::pair<int, int>, V3<double>> keep;
    for (auto &kv : s->shist) {
        const int k = kv.first.second;
        if (k < count && k < (int)s->surf.size() && std::memcmp(&s->surf[k], &next[k], sizeof(Surface)) == 0)
            keep[kv.first] = kv.second;
    }
    s->shist.swap(keep);
    s->surf = next;
}

/* The contact geometry of one sphere and one surface record (9 doubles as
 * above): returns 1 in contact, with out = (distance, n_x, n_y, n_z). */
int orc_surface_contact(const double *desc, double x, double y, double z, double r, double *out) {
    Surface w{(int)desc[0], (int)desc[1], desc[2], desc[3], desc[4], desc[5], desc[6], desc[7], desc[8]};
    double d;
    V3<double> n;
    if (!surface_contact(w, x, y, z, r, d, n)) return 0;
    out[0] = d; out[1] = n.x; out[2] = n.y; out[3] = n.z;
    return 1;
}

/* Surface history: (id, surface index, xi). */
long orc_surface_history(void *h, int *id, int *k, double *xi, long cap) {
    SimD *s = (SimD *)h;
    long q = 0;
    for (auto &kv : s->shist) {
        if (q < cap) {
            id[q] = kv.first.first; k[q] = kv.first.second;
            xi[3 * q] = kv.second.x; xi[3 * q + 1] = kv.second.y; xi[3 * q + 2] = kv.second.z;
        }
        ++q;
    }
    return q;
}

void orc_set_surface_history(void *h, long count, const int *id, const int *k, const double *xi) {
    SimD *s = (SimD *)h;
    s->shist.clear();
    for (long q = 0; q < count; ++q) s->shist[{id[q], k[q]}] = {xi[3 * q], xi[3 * q + 1], xi[3 * q + 2]};
}

/* External force on every particle, (n, 3) in input order, added after the
 * wall term at every force evaluation; null removes it. */
void orc_set_external(void *h, const double *f) {
    SimD *s = (SimD *)h;
    if (!f) { s->fext.clear(); return; }
    s->fext.resize(s->p.size());
    for (size_t i = 0; i < s->p.size(); ++i) s->fext[i] = {f[3 * i], f[3 * i + 1], f[3 * i + 2]};
}

/* Contact forces of the current state without touching the history (as a
 * force evaluation without history update): for every unordered pair in
 * contact, ids (lo < hi), the branch vector d = x_lo - x_hi (minimum image)
 * and the force on lo (the force on hi is its negative).  Returns the count;
 * arrays of cap entries (d, f: [cap][3]) may be null. */
long orc_pair_forces(void *h, int *lo, int *hi, double *d, double *f, long cap) {
    SimD *s = (SimD *)h;
    const Config &c = s->cfg;
    std::vector<std::pair<int, int>> cand;
    grid_pairs(*s, 0.0, cand);
    long k = 0;
    for (auto &pr : cand) {
        const Particle<double> &a = s->p[pr.first];
        const Particle<double> &b = s->p[pr.second];
        auto it = s->hist.find({a.id, b.id});
        V3<double> xi = it == s->hist.end() ? V3<double>{0.0, 0.0, 0.0} : it->second;
        V3<double> fo, ft, n;
        if (!contact(*s, a, &b, xi, false, fo, ft, n, (PairRecord<double> *)nullptr)) continue;
        if (k < cap) {
            if (lo) lo[k] = a.id;
            if (hi) hi[k] = b.id;
            if (d) {
                d[3 * k] = min_image(a.x.x - b.x.x, c.hi[0] - c.lo[0], c.periodic[0]);
                d[3 * k + 1] = min_image(a.x.y - b.x.y, c.hi[1] - c.lo[1], c.periodic[1]);
                d[3 * k + 2] = min_image(a.x.z - b.x.z, c.hi[2] - c.lo[2], c.periodic[2]);
            }
            if (f) { f[3 * k] = fo.x; f[3 * k + 1] = fo.y; f[3 * k + 2] = fo.z; }
        }
        ++k;
    }
    return k;
}

/* ------------------------------------------------ forward-mode tangents */

/* Same simulation with dual numbers: derivative directions are
 * (E_0, E_1, e_0, e_1, mu_0, mu_1); types beyond 2 carry no tangent. */
void *orc_tan_new(const orc_config *cfg, int n, const double *x, const double *v, const double *w, const double *r,
                  const int *type, const int *id) {
    SimT *s = make<Dual>(cfg, n, x, v, w, r, type, id);
    for (int t = 0; t < cfg->ntypes && t < 2; ++t) {
        s->E[t].d[0 + t] = 1.0;
        s->e[t].d[2 + t] = 1.0;
        s->mu[t].d[4 + t] = 1.0;
    }
    return s;
}
/* Re-seed tangent direction k (0..5) along the initial state: x += eps dx,
 * v += eps dv, w += eps dw ((n,3) arrays in input order; null = zero), with
 * no parameter moving in that direction. */
void orc_tan_seed_state(void *h, int k, const double *dx, const double *dv, const double *dw) {
    SimT *s = (SimT *)h;
    if (k < 0 || k >= NDIR) return;
    for (int t = 0; t < 4; ++t) { s->E[t].d[k] = 0.0; s->e[t].d[k] = 0.0; s->mu[t].d[k] = 0.0; }
    for (size_t i = 0; i < s->p.size(); ++i) {
        Particle<Dual> &q = s->p[i];
        V3<Dual> *vec[3] = {&q.x, &q.v, &q.w};
        const double *src[3] = {dx, dv, dw};
        for (int a = 0; a < 3; ++a) {
            Dual *c3[3] = {&vec[a]->x, &vec[a]->y, &vec[a]->z};
            for (int c = 0; c < 3; ++c) c3[c]->d[k] = src[a] ? src[a][3 * i + c] : 0.0;
        }
    }
}
void orc_tan_free(void *h) { delete (SimT *)h; }
void orc_tan_forces(void *h, int update_history) { forces(*(SimT *)h, update_history != 0); }
void orc_tan_step(void *h, int nsteps) { step(*(SimT *)h, nsteps); }

/* Value and tangent of one per-particle vector: which = 0..4 for x, v, w, f, t;
 * val[n*3], tan[n*3*6] (direction fastest).  Either pointer may be null. */
void orc_tan_get_ext(void *h, int which, double *val, double *tan) {
    SimT *s = (SimT *)h;
    for (size_t i = 0; i < s->p.size(); ++i) {
        const Particle<Dual> &q = s->p[i];
        const V3<Dual> *vec[5] = {&q.x, &q.v, &q.w, &q.f, &q.t};
        const V3<Dual> &u = *vec[which < 0 || which > 4 ? 0 : which];
        const Dual *c3[3] = {&u.x, &u.y, &u.z};
        for (int c = 0; c < 3; ++c) {
            if (val) val[3 * i + c] = c3[c]->v;
            if (tan)
                for (int k = 0; k < NDIR; ++k) tan[(3 * i + c) * NDIR + k] = c3[c]->d[k];
        }
    }
}

/* Values and tangents of x and v: val[n*3], tan[n*3*6] (direction fastest). */
void orc_tan_get(void *h, double *xv, double *xt, double *vv, double *vt) {
    SimT *s = (SimT *)h;
    for (size_t i = 0; i < s->p.size(); ++i) {
        const Particle<Dual> &q = s->p[i];
        const Dual *X[3] = {&q.x.x, &q.x.y, &q.x.z};
        const Dual *Vv[3] = {&q.v.x, &q.v.y, &q.v.z};
        for (int c = 0; c < 3; ++c) {
            if (xv) xv[3 * i + c] = X[c]->v;
            if (vv) vv[3 * i + c] = Vv[c]->v;
            for (int k = 0; k < NDIR; ++k) {
                if (xt) xt[(3 * i + c) * NDIR + k] = X[c]->d[k];
                if (vt) vt[(3 * i + c) * NDIR + k] = Vv[c]->d[k];
            }
        }
    }
}

}  // extern "C"
