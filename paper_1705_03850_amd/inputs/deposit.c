/*
 * deposit.c -- geometric sequential deposition ("drop and roll") of spheres
 * onto a flat floor at z = 0 in a box that is periodic in x and y.
 *
 * This is an input generator.  It contains no contact mechanics: each new
 * sphere falls vertically, then rolls without friction along the surfaces of
 * the spheres it touches (steepest descent of its height, the classic
 * Visscher-Bolsterli construction), and comes to rest when gravity is carried
 * by compressive contacts on three spheres, or when it touches the floor.
 * Every random number (drop position, tie-break azimuth) is drawn by the
 * caller and passed in, so the output is a pure function of the inputs.
 *
 * Build: gcc -O2 -fPIC -shared deposit.c -o libdeposit.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double Lx, Ly, hx, hy, h;
    int ncx, ncy, ncz;
    int *head;   /* [ncx*ncy*ncz] first sphere in cell, -1 = empty */
    int *next;   /* [n] next sphere in the same cell              */
    double *x, *y, *z, *r;
    int n;
    int *stamp;  /* [n] de-duplication marks for cell queries      */
    int stamp_val;
    double zmax; /* highest centre placed so far                  */
    double rmax;
} Pile;

static double wrap_d(double d, double L) {
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

static double wrap_p(double p, double L) {
    p = fmod(p, L);
    if (p < 0.0) p += L;
    if (p >= L) p = 0.0;
    return p;
}

static int cell_of(const Pile *P, double x, double y, double z, int *cx, int *cy, int *cz) {
    int ix = (int)floor(x / P->hx), iy = (int)floor(y / P->hy), iz = (int)floor(z / P->h);
    ix = ((ix % P->ncx) + P->ncx) % P->ncx;
    iy = ((iy % P->ncy) + P->ncy) % P->ncy;
    if (iz < 0) iz = 0;
    if (iz >= P->ncz) iz = P->ncz - 1;
    *cx = ix; *cy = iy; *cz = iz;
    return (iz * P->ncy + iy) * P->ncx + ix;
}

static void insert(Pile *P, int k) {
    int cx, cy, cz;
    int c = cell_of(P, P->x[k], P->y[k], P->z[k], &cx, &cy, &cz);
    P->next[k] = P->head[c];
    P->head[c] = k;
    if (P->z[k] > P->zmax) P->zmax = P->z[k];
}

/* Collect the spheres whose centres may lie inside the axis-aligned box
 * [x0,x1]x[y0,y1]x[z0,z1] (x,y unwrapped, periodic).  Returns the count. */
static int query_box(Pile *P, double x0, double x1, double y0, double y1, double z0, double z1,
                     int *out, int cap) {
    int ix0 = (int)floor(x0 / P->hx), ix1 = (int)floor(x1 / P->hx);
    int iy0 = (int)floor(y0 / P->hy), iy1 = (int)floor(y1 / P->hy);
    int iz0 = (int)floor(z0 / P->h), iz1 = (int)floor(z1 / P->h);
    if (ix1 - ix0 >= P->ncx) { ix0 = 0; ix1 = P->ncx - 1; }
    if (iy1 - iy0 >= P->ncy) { iy0 = 0; iy1 = P->ncy - 1; }
    if (iz0 < 0) iz0 = 0;
    if (iz1 >= P->ncz) iz1 = P->ncz - 1;
    if (iz0 > iz1) return 0;
    P->stamp_val++;
    int m = 0;
    for (int iz = iz0; iz <= iz1; ++iz)
        for (int iy = iy0; iy <= iy1; ++iy)
            for (int ix = ix0; ix <= ix1; ++ix) {
                int cx = ((ix % P->ncx) + P->ncx) % P->ncx;
                int cy = ((iy % P->ncy) + P->ncy) % P->ncy;
                for (int k = P->head[(iz * P->ncy + cy) * P->ncx + cx]; k >= 0; k = P->next[k]) {
                    if (P->stamp[k] == P->stamp_val) continue;
                    P->stamp[k] = P->stamp_val;
                    if (m < cap) out[m++] = k;
                }
            }
    return m;
}

/* Vector from sphere k's nearest periodic image to point p. */
static void rel(const Pile *P, int k, const double p[3], double d[3]) {
    d[0] = wrap_d(p[0] - P->x[k], P->Lx);
    d[1] = wrap_d(p[1] - P->y[k], P->Ly);
    d[2] = p[2] - P->z[k];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* Path p(t) = c + R (cos t e1 + sin t e2), travelling from t0 in direction dir
 * (+1/-1) over a parameter length slen.  First entry (from outside) into the
 * ball |p - q| < rho.  Returns the travelled length s, or -1. */
static double first_entry(const double c[3], double R, const double e1[3], const double e2[3], double t0,
                          int dir, double slen, const double q[3], double rho) {
    double cq[3] = {c[0] - q[0], c[1] - q[1], c[2] - q[2]};
    double cq2 = dot3(cq, cq);
    if (cq2 >= (R + rho) * (R + rho)) return -1.0; /* ball out of reach of the whole circle */
    double a = R * dot3(cq, e1), b = R * dot3(cq, e2);
    double K = 0.5 * (rho * rho - cq2 - R * R);
    /* already touching (or overlapping by rounding) and moving inwards: event now */
    if (a * cos(t0) + b * sin(t0) - K < 1e-9 * rho * rho &&
        dir * (-a * sin(t0) + b * cos(t0)) < 0.0) return 0.0;
    double M = hypot(a, b);
    if (M <= 0.0 || fabs(K) > M) return -1.0;
    double phi = atan2(b, a), w = acos(K / M);
    double best = -1.0;
    for (int s = -1; s <= 1; s += 2) {
        double tr = phi + s * w;
        double ds = (tr - t0) * dir;
        ds = fmod(ds, 2.0 * M_PI);
        if (ds < 0.0) ds += 2.0 * M_PI;
        if (ds <= 1e-12 || ds > slen) continue;
        /* entering: a cos t + b sin t decreasing along the travel direction */
        double deriv = dir * (-a * sin(tr) + b * cos(tr));
        if (deriv >= 0.0) continue;
        if (best < 0.0 || ds < best) best = ds;
    }
    return best;
}

/* Same path, first time the height reaches zf from above. */
static double first_floor(const double c[3], double R, const double e1[3], const double e2[3], double t0,
                          int dir, double slen, double zf) {
    double a = R * e1[2], b = R * e2[2];
    double K = zf - c[2];
    if (a * cos(t0) + b * sin(t0) - K < 1e-9 * zf && dir * (-a * sin(t0) + b * cos(t0)) < 0.0) return 0.0;
    double M = hypot(a, b);
    if (M <= 0.0 || fabs(K) > M) return -1.0;
    double phi = atan2(b, a), w = acos(K / M);
    double best = -1.0;
    for (int s = -1; s <= 1; s += 2) {
        double tr = phi + s * w;
        double ds = (tr - t0) * dir;
        ds = fmod(ds, 2.0 * M_PI);
        if (ds < 0.0) ds += 2.0 * M_PI;
        if (ds <= 1e-12 || ds > slen) continue;
        double deriv = dir * (-a * sin(tr) + b * cos(tr));
        if (deriv >= 0.0) continue;
        if (best < 0.0 || ds < best) best = ds;
    }
    return best;
}

/* Solve the 2x2 / 3x3 systems sum_k alpha_k n_k = g (least squares for 2). */
static void alphas2(const double nA[3], const double nB[3], double out[2]) {
    const double g[3] = {0.0, 0.0, -1.0};
    double c = dot3(nA, nB), gA = dot3(g, nA), gB = dot3(g, nB);
    double det = 1.0 - c * c;
    if (fabs(det) < 1e-14) { out[0] = out[1] = 1.0; return; }
    out[0] = (gA - c * gB) / det;
    out[1] = (gB - c * gA) / det;
}

static int alphas3(const double n0[3], const double n1[3], const double n2[3], double out[3]) {
    const double g[3] = {0.0, 0.0, -1.0};
    double c12[3], c20[3], c01[3];
    cross3(n1, n2, c12); cross3(n2, n0, c20); cross3(n0, n1, c01);
    double det = dot3(n0, c12);
    if (fabs(det) < 1e-14) return 0;
    out[0] = dot3(g, c12) / det;
    out[1] = dot3(g, c20) / det;
    out[2] = dot3(g, c01) / det;
    return 1;
}

/* Active contact set for a sphere touching the given supports (unit normals
 * pointing from each support to the sphere), frictionless, under g = -z.
 * Returns the number of supports kept (0 = free fall) and their positions in
 * keep[].  A kept pair must have both contacts in compression and its
 * downhill motion must not push into a released support; a kept single must
 * be pressed by gravity and roll away from the released ones. */
static int active_set(const double *const *nv, int m, int keep[3]) {
    const double g[3] = {0.0, 0.0, -1.0};
    if (m == 3) {
        double al3[3];
        if (alphas3(nv[0], nv[1], nv[2], al3) && al3[0] <= 0.0 && al3[1] <= 0.0 && al3[2] <= 0.0) {
            keep[0] = 0; keep[1] = 1; keep[2] = 2;
            return 3;
        }
    }
    if (m >= 2) {
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) {
                double al[2];
                alphas2(nv[i], nv[j], al);
                if (al[0] > 0.0 || al[1] > 0.0) continue;
                double gt[3];
                for (int d = 0; d < 3; ++d) gt[d] = g[d] - al[0] * nv[i][d] - al[1] * nv[j][d];
                int ok = 1;
                for (int k = 0; k < m; ++k)
                    if (k != i && k != j && dot3(gt, nv[k]) < 0.0) ok = 0;
                if (!ok) continue;
                keep[0] = i; keep[1] = j;
                return 2;
            }
    }
    for (int i = 0; i < m; ++i) {
        double gi = dot3(g, nv[i]);
        if (gi >= 0.0) continue;
        double di[3];
        for (int d = 0; d < 3; ++d) di[d] = g[d] - gi * nv[i][d];
        int ok = 1;
        for (int k = 0; k < m; ++k)
            if (k != i && dot3(di, nv[k]) < 0.0) ok = 0;
        if (!ok) continue;
        keep[0] = i;
        return 1;
    }
    return 0;
}

enum { ST_DROP, ST_ROLL1, ST_ROLL2, ST_REST };

#define QCAP 4096

/*
 * Deposit n spheres with radii r[k] (already scaled by the caller) at drop
 * positions (dx[k], dy[k]) in [0,Lx)x[0,Ly).  az[k] in [0, 2 pi) breaks the
 * tie when a sphere lands exactly on top of another.  zcap bounds the cell
 * grid height (spheres above it share the top layer, still correct).
 * Writes centres to (x, y, z).  Returns the number of spheres that hit the
 * event limit and were left where they stopped (diagnostic).
 */
int deposit(int n, const double *r, const double *dx, const double *dy, const double *az, double Lx,
            double Ly, double zcap, double *x, double *y, double *z) {
    Pile P;
    memset(&P, 0, sizeof P);
    double rmax = 0.0;
    for (int k = 0; k < n; ++k) rmax = r[k] > rmax ? r[k] : rmax;
    P.rmax = rmax;
    P.Lx = Lx; P.Ly = Ly;
    P.ncx = (int)floor(Lx / (2.0 * rmax));
    P.ncy = (int)floor(Ly / (2.0 * rmax));
    if (P.ncx < 1) P.ncx = 1;
    if (P.ncy < 1) P.ncy = 1;
    /* cells tile the periodic box exactly, so an image shift is a whole number of cells */
    P.hx = Lx / P.ncx;
    P.hy = Ly / P.ncy;
    P.h = 2.0 * rmax;
    P.ncz = (int)ceil(zcap / P.h) + 1;
    size_t ncell = (size_t)P.ncx * P.ncy * P.ncz;
    P.head = (int *)malloc(ncell * sizeof(int));
    for (size_t c = 0; c < ncell; ++c) P.head[c] = -1;
    P.next = (int *)malloc((size_t)n * sizeof(int));
    P.stamp = (int *)calloc((size_t)n, sizeof(int));
    P.x = x; P.y = y; P.z = z; P.r = (double *)r;
    P.n = 0;
    P.zmax = 0.0;
    int *cand = (int *)malloc(QCAP * sizeof(int));
    int stuck = 0;

    for (int k = 0; k < n; ++k) {
        double rp = r[k];
        double p[3] = {wrap_p(dx[k], Lx), wrap_p(dy[k], Ly), P.zmax + 2.0 * rmax + rp + 1e-9};
        int state = ST_DROP;
        int A = -1, B = -1, excl[3] = {-1, -1, -1};
        int events = 0;
        while (state != ST_REST) {
            if (++events > 64) { stuck++; break; }
            if (state == ST_DROP) {
                /* fall vertically from p: scan cell layers from the top down and
                 * stop once no lower layer can hold a higher landing point */
                double best = rp;
                int hit = -1;
                double reach = rp + rmax;
                int iztop = (int)floor((p[2] + reach) / P.h);
                if (iztop >= P.ncz) iztop = P.ncz - 1;
                for (int iz = iztop; iz >= 0; --iz) {
                    if (iz < P.ncz - 1 && best >= (iz + 1) * P.h + reach) break;
                    double zl = iz * P.h + 0.5 * P.h;
                    int m = query_box(&P, p[0] - reach, p[0] + reach, p[1] - reach, p[1] + reach, zl, zl,
                                      cand, QCAP);
                    for (int i = 0; i < m; ++i) {
                        int j = cand[i];
                        if (j == excl[0] || j == excl[1] || j == excl[2]) continue;
                        double d[3];
                        rel(&P, j, p, d);
                        double rho = rp + r[j];
                        double h2 = d[0] * d[0] + d[1] * d[1];
                        if (h2 >= rho * rho) continue;
                        double zh = P.z[j] + sqrt(rho * rho - h2);
                        if (zh > p[2] + 1e-12) continue; /* above the start: not on the way down */
                        if (zh > best) { best = zh; hit = j; }
                    }
                }
                p[2] = best;
                excl[0] = excl[1] = excl[2] = -1;
                if (hit < 0) { state = ST_REST; break; }
                A = hit;
                state = ST_ROLL1;
            } else if (state == ST_ROLL1) {
                double a[3] = {P.x[A], P.y[A], P.z[A]};
                double u[3];
                rel(&P, A, p, u);
                double rhoA = rp + r[A];
                double uh = hypot(u[0], u[1]);
                double eh[3];
                if (uh < 1e-12 * rhoA) {
                    eh[0] = cos(az[k]); eh[1] = sin(az[k]); eh[2] = 0.0;
                } else {
                    eh[0] = u[0] / uh; eh[1] = u[1] / uh; eh[2] = 0.0;
                }
                double ez[3] = {0.0, 0.0, 1.0};
                double t0 = atan2(uh, u[2]); /* polar angle from +z */
                double slen = 0.5 * M_PI - t0;
                if (slen <= 0.0) { /* at or below the equator: falls off */
                    excl[0] = A; state = ST_DROP; continue;
                }
                /* centre of the path: a (in p's frame) */
                double c[3] = {p[0] - u[0], p[1] - u[1], p[2] - u[2]};
                (void)a;
                double best = slen, ev = 0; /* ev: 0 equator, 1 sphere, 2 floor */
                int hitk = -1;
                double reach = rhoA + rp + rmax;
                int m = query_box(&P, c[0] - reach, c[0] + reach, c[1] - reach, c[1] + reach,
                                  c[2] - reach, c[2] + reach, cand, QCAP);
                for (int i = 0; i < m; ++i) {
                    int j = cand[i];
                    if (j == A) continue;
                    double q[3], dq[3];
                    rel(&P, j, c, dq);
                    q[0] = c[0] - dq[0]; q[1] = c[1] - dq[1]; q[2] = c[2] - dq[2];
                    double s = first_entry(c, rhoA, ez, eh, t0, +1, slen, q, rp + r[j]);
                    if (s >= 0.0 && s < best) { best = s; ev = 1; hitk = j; }
                }
                double sf = first_floor(c, rhoA, ez, eh, t0, +1, slen, rp);
                if (sf >= 0.0 && sf < best) { best = sf; ev = 2; }
                double t = t0 + best;
                for (int d = 0; d < 3; ++d) p[d] = c[d] + rhoA * (cos(t) * ez[d] + sin(t) * eh[d]);
                if (ev == 2) { state = ST_REST; break; }
                if (ev == 0) { excl[0] = A; state = ST_DROP; continue; }
                B = hitk;
                state = ST_ROLL2;
            } else { /* ST_ROLL2 on A and B */
                double uA[3], uB[3];
                rel(&P, A, p, uA);
                rel(&P, B, p, uB);
                double rhoA = rp + r[A], rhoB = rp + r[B];
                double nA[3] = {uA[0] / rhoA, uA[1] / rhoA, uA[2] / rhoA};
                double nB[3] = {uB[0] / rhoB, uB[1] / rhoB, uB[2] / rhoB};
                {
                    const double *nv[2] = {nA, nB};
                    int keep[3], ids[2] = {A, B};
                    int na = active_set(nv, 2, keep);
                    if (na == 0) { excl[0] = A; excl[1] = B; state = ST_DROP; continue; }
                    if (na == 1) { A = ids[keep[0]]; B = -1; state = ST_ROLL1; continue; }
                }
                /* circle of points at distance rhoA from a and rhoB from b (images near p) */
                double a[3] = {p[0] - uA[0], p[1] - uA[1], p[2] - uA[2]};
                double b[3] = {p[0] - uB[0], p[1] - uB[1], p[2] - uB[2]};
                double dab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
                double D = norm3(dab);
                double e[3] = {dab[0] / D, dab[1] / D, dab[2] / D};
                double tc = (D * D + rhoA * rhoA - rhoB * rhoB) / (2.0 * D);
                double hc2 = rhoA * rhoA - tc * tc;
                if (hc2 <= 0.0) { state = ST_REST; break; }
                double hc = sqrt(hc2);
                double c[3] = {a[0] + tc * e[0], a[1] + tc * e[1], a[2] + tc * e[2]};
                double g1[3] = {e[2] * e[0], e[2] * e[1], e[2] * e[2] - 1.0}; /* -z + e_z e */
                double gl = norm3(g1);
                if (gl < 1e-12) { state = ST_REST; break; } /* horizontal circle */
                double e1[3] = {g1[0] / gl, g1[1] / gl, g1[2] / gl};
                double e2[3];
                cross3(e, e1, e2);
                double pc[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
                double psi0 = atan2(dot3(pc, e2), dot3(pc, e1));
                int dir = psi0 > 0.0 ? -1 : +1;
                double slen = fabs(psi0);
                double best = slen;
                int ev = 0, hitk = -1;
                if (slen > 1e-14) {
                    double reach = rhoA + rp + rmax;
                    int m = query_box(&P, a[0] - reach, a[0] + reach, a[1] - reach, a[1] + reach,
                                      a[2] - reach, a[2] + reach, cand, QCAP);
                    for (int i = 0; i < m; ++i) {
                        int j = cand[i];
                        if (j == A || j == B) continue;
                        double dq[3], q[3];
                        rel(&P, j, c, dq);
                        q[0] = c[0] - dq[0]; q[1] = c[1] - dq[1]; q[2] = c[2] - dq[2];
                        double s = first_entry(c, hc, e1, e2, psi0, dir, slen, q, rp + r[j]);
                        if (s >= 0.0 && s < best) { best = s; ev = 1; hitk = j; }
                    }
                    double sf = first_floor(c, hc, e1, e2, psi0, dir, slen, rp);
                    if (sf >= 0.0 && sf < best) { best = sf; ev = 2; }
                }
                double t = psi0 + dir * best;
                for (int d = 0; d < 3; ++d) p[d] = c[d] + hc * (cos(t) * e1[d] + sin(t) * e2[d]);
                if (ev == 2) { state = ST_REST; break; }
                if (ev == 0) {
                    /* lowest point of the circle: balanced if both contacts compress */
                    rel(&P, A, p, uA);
                    rel(&P, B, p, uB);
                    for (int d = 0; d < 3; ++d) { nA[d] = uA[d] / rhoA; nB[d] = uB[d] / rhoB; }
                    const double *nv[2] = {nA, nB};
                    int keep[3], ids[2] = {A, B};
                    int na = active_set(nv, 2, keep);
                    if (na == 2) { state = ST_REST; break; }
                    if (na == 0) { excl[0] = A; excl[1] = B; state = ST_DROP; continue; }
                    A = ids[keep[0]]; B = -1;
                    state = ST_ROLL1;
                    continue;
                }
                /* third contact C: stable when all three contacts compress */
                int C = hitk;
                double uC[3], nC[3];
                rel(&P, A, p, uA);
                rel(&P, B, p, uB);
                rel(&P, C, p, uC);
                double rhoC = rp + r[C];
                for (int d = 0; d < 3; ++d) { nA[d] = uA[d] / rhoA; nB[d] = uB[d] / rhoB; nC[d] = uC[d] / rhoC; }
                const double *nv[3] = {nA, nB, nC};
                int keep[3], ids[3] = {A, B, C};
                int na = active_set(nv, 3, keep);
                if (na == 3) { state = ST_REST; break; }
                if (na == 0) { excl[0] = A; excl[1] = B; excl[2] = C; state = ST_DROP; continue; }
                if (na == 2) { A = ids[keep[0]]; B = ids[keep[1]]; state = ST_ROLL2; }
                else { A = ids[keep[0]]; B = -1; state = ST_ROLL1; }
            }
        }
        x[k] = wrap_p(p[0], Lx);
        y[k] = wrap_p(p[1], Ly);
        z[k] = p[2];
        P.n = k + 1;
        insert(&P, k);
    }
    free(cand);
    free(P.head);
    free(P.next);
    free(P.stamp);
    return stuck;
}
