// dem_adjoint.hip -- kernels of the reverse-mode rollout (gradients of a
// trajectory with respect to the contact-law parameters of Eq. (3)-(6)).
//
// One group of G lanes per particle (4 or 8), like the force pass of the step.  The
// recompute kernel repeats the step's arithmetic in the step's order (slots
// summed in ascending neighbour id, then the wall), so it reproduces the
// forward trajectory bit for bit.  The reverse kernel evaluates, for every
// slot of a particle's row, the adjoint of the pair with the seeds of both
// directed contacts combined (the force seed of i minus that of j, the torque
// seeds r_i T_i + r_j T_j, the slot's history adjoint), keeps the adjoints of
// its own particle's inputs and writes its own slot's history adjoint: the
// partner computes the mirror image of the same pair, so there are no
// scatters and no atomics.  Each unordered pair is thus seen twice, and its
// coefficient adjoint is counted with a factor 1/2.
#include "dem_adjoint.h"

namespace dem {

namespace {

constexpr int kABlock = 256;
// Waves per SIMD the reverse kernel is compiled for: 2 caps it at 256
// registers (a few spill to scratch), which ran the chute backward 11 % faster
// than one wave with no spills.
constexpr int kAdjReverseWaves = 2;

// Sum over the G lanes of a group, in lane order.
template <int G>
__device__ inline double group_sum(double v, int gbase) {
    double s = __shfl(v, gbase);
#pragma unroll
    for (int l = 1; l < G; ++l) s = s + __shfl(v, gbase + l);
    return s;
}

int adj_grid(int64_t n, int lanes) {
    int64_t g = (n * lanes + kABlock - 1) / kABlock;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    return (int)g;
}

int flat_grid(int64_t n) {
    int64_t g = (n + kABlock - 1) / kABlock;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

}  // namespace

// ------------------------------------------------------------ history form

__global__ void k_adj_expand(AArgs a, const D4 *xi, const uint64_t *mask, const double *xiw, D4 *hout, D4 *hwout) {
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t m = mask[i];
        const int cnt = a.cnt[i];
        for (int q = 0; q < cnt; ++q) {
            D4 h = {0.0, 0.0, 0.0, 0.0};
            if ((m >> q) & 1ull) {
                const D4 v = xi[i * a.kmax + q];
                h = D4{v.x, v.y, v.z, 0.0};
            }
            hout[i * a.kslots + q] = h;
        }
        hwout[i] = (m & kWallBit) ? D4{xiw[i], xiw[n + i], xiw[2 * n + i], 0.0} : D4{0.0, 0.0, 0.0, 0.0};
    }
}

// ------------------------------------------------------------ recompute

// The system's pair coefficients, read by every contact: in LDS (the reverse
// kernel, at its register limit, reads them from global memory: the LDS copy
// cost it spills).
__shared__ PairCoef adj_coef[kMaxTypes * kMaxTypes];

__device__ __forceinline__ void load_adj_coef(const AArgs &a) {
    for (int k = threadIdx.x; k < a.ntypes * a.ntypes; k += blockDim.x) adj_coef[k] = a.coef[k];
    __syncthreads();
}

template <int G, int MODE>
__global__ void __launch_bounds__(kABlock, 4) k_adj_forward(AArgs a) {
    int64_t step = 0;
    if (MODE != 0) {
        step = a.flags->step_base + a.k;
        if (a.flags->abort_at <= step) return;
    }
    bool need = false, bad = false;
    const int64_t n = a.n;
    const int64_t ks = a.kslots;
    const SysDesc s = uniform_sys(a.sys);
    load_adj_coef(a);
    const int g = threadIdx.x % G;
    const int gbase = (threadIdx.x % warpSize) / G * G;
    const uint64_t gmask = (1ull << G) - 1;
    const int64_t ppb = blockDim.x / G;
    for (int64_t i0 = (int64_t)blockIdx.x * ppb; i0 < n; i0 += (int64_t)gridDim.x * ppb) {
        const int64_t i = i0 + threadIdx.x / G;
        if (i >= n) continue;
        const D4 pi = a.pos[i], vi = a.vel[i], si = a.spin[i];
        const int ti = (int)si.w & 15;
        const double ri = pi.w, mi = vi.w;
        double Fx = mi * s.g[0], Fy = mi * s.g[1], Fz = mi * s.g[2];
        double Tx = 0.0, Ty = 0.0, Tz = 0.0;
        const int cnt = a.cnt[i];
        for (int c0 = 0; c0 < cnt; c0 += G) {
            const int q = c0 + g;
            const bool valid = q < cnt;
            const int64_t slot = i * ks + q;
            const int32_t j = valid ? a.nbr[q * n + i] : (int32_t)i;
            const D4 pj = a.pos[j];
            ContactIn c;
            c.dx = min_image(pi.x - pj.x, s.L[0], s.hL[0], s.periodic[0]);
            c.dy = min_image(pi.y - pj.y, s.L[1], s.hL[1], s.periodic[1]);
            c.dz = min_image(pi.z - pj.z, s.L[2], s.hL[2], s.periodic[2]);
            c.ra = ri;
            c.rb = pj.w;
            const double rs = c.ra + c.rb;
            double fx = 0.0, fy = 0.0, fz = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
            bool hit = false;
            D4 hnew = {0.0, 0.0, 0.0, 0.0};
            if (valid && c.dx * c.dx + c.dy * c.dy + c.dz * c.dz < rs * rs) {
                const D4 vj = a.vel[j], sj = a.spin[j];
                const D4 h = a.hin[slot];
                double hx = h.x, hy = h.y, hz = h.z;
                c.ma = mi; c.mb = vj.w;
                c.vrx = vi.x - vj.x; c.vry = vi.y - vj.y; c.vrz = vi.z - vj.z;
                c.wsx = ri * si.x + pj.w * sj.x;
                c.wsy = ri * si.y + pj.w * sj.y;
                c.wsz = ri * si.z + pj.w * sj.z;
                const PairCoef pc = adj_coef[ti * a.ntypes + ((int)sj.w & 15)];
                double ftx, fty, ftz, nx, ny, nz, fn;
                if (contact_force(c, false, pc, s.dt, true, hx, hy, hz, fx, fy, fz, ftx, fty, ftz, nx, ny, nz, fn)) {
                    hit = true;
                    tx = -(ri * (ny * ftz - nz * fty));
                    ty = -(ri * (nz * ftx - nx * ftz));
                    tz = -(ri * (nx * fty - ny * ftx));
                    hnew = D4{hx, hy, hz, 0.0};
                }
            }
            if (valid) a.hout[slot] = hnew;
            uint64_t b = (__ballot(hit) >> gbase) & gmask;
            while (b) {
                const int src = gbase + __builtin_ctzll(b);
                b &= b - 1;
                Fx = Fx + __shfl(fx, src);
                Fy = Fy + __shfl(fy, src);
                Fz = Fz + __shfl(fz, src);
                Tx = Tx + __shfl(tx, src);
                Ty = Ty + __shfl(ty, src);
                Tz = Tz + __shfl(tz, src);
            }
        }
        D4 hw = {0.0, 0.0, 0.0, 0.0};
        if (s.wall && pi.z < ri) {
            ContactIn c;
            c.dx = 0.0; c.dy = 0.0; c.dz = pi.z;
            c.ra = ri; c.rb = 0.0; c.ma = mi; c.mb = 0.0;
            c.vrx = vi.x; c.vry = vi.y; c.vrz = vi.z;
            c.wsx = ri * si.x; c.wsy = ri * si.y; c.wsz = ri * si.z;
            const PairCoef pc = adj_coef[ti * a.ntypes + ti];
            const D4 h = a.hwin[i];
            double hx = h.x, hy = h.y, hz = h.z;
            double fx, fy, fz, ftx, fty, ftz, nx, ny, nz, fn;
            if (contact_force(c, true, pc, s.dt, true, hx, hy, hz, fx, fy, fz, ftx, fty, ftz, nx, ny, nz, fn)) {
                Fx = Fx + fx; Fy = Fy + fy; Fz = Fz + fz;
                Tx = Tx + -(ri * (ny * ftz - nz * fty));
                Ty = Ty + -(ri * (nz * ftx - nx * ftz));
                Tz = Tz + -(ri * (nx * fty - ny * ftx));
                hw = D4{hx, hy, hz, 0.0};
            }
        }
        if (g != 0) continue;
        a.hwout[i] = hw;
        const D2 im = a.im[i];
        double vx = vi.x + s.hdt * (Fx * im.a), vy = vi.y + s.hdt * (Fy * im.a), vz = vi.z + s.hdt * (Fz * im.a);
        double wx = si.x + s.hdt * (Tx * im.b), wy = si.y + s.hdt * (Ty * im.b), wz = si.z + s.hdt * (Tz * im.b);
        if (MODE == 2) {
            a.f[i] = Fx; a.f[n + i] = Fy; a.f[2 * n + i] = Fz;
            a.t[i] = Tx; a.t[n + i] = Ty; a.t[2 * n + i] = Tz;
            a.x[i] = pi.x; a.x[n + i] = pi.y; a.x[2 * n + i] = pi.z;
            a.v[i] = vx; a.v[n + i] = vy; a.v[2 * n + i] = vz;
            a.w[i] = wx; a.w[n + i] = wy; a.w[2 * n + i] = wz;
            continue;
        }
        vx = vx + s.hdt * (Fx * im.a); vy = vy + s.hdt * (Fy * im.a); vz = vz + s.hdt * (Fz * im.a);
        wx = wx + s.hdt * (Tx * im.b); wy = wy + s.hdt * (Ty * im.b); wz = wz + s.hdt * (Tz * im.b);
        const double x = wrap_axis(pi.x + s.dt * vx, s, 0);
        const double y = wrap_axis(pi.y + s.dt * vy, s, 1);
        const double z = wrap_axis(pi.z + s.dt * vz, s, 2);
        if (MODE == 1) {
            // displacement since the last build and the rebuild request, as in the fused step
            const double ddx = a.disp[i] + s.dt * vx;
            const double ddy = a.disp[n + i] + s.dt * vy;
            const double ddz = a.disp[2 * n + i] + s.dt * vz;
            a.disp[i] = ddx; a.disp[n + i] = ddy; a.disp[2 * n + i] = ddz;
            double dsq = 0.0;
            dsq += ddx * ddx;
            dsq += ddy * ddy;
            dsq += ddz * ddz;
            if (!(dsq <= s.disp_thr2)) need = true;
            if (!isfinite(x + y + z + vx + vy + vz)) bad = true;
        }
        a.pos_o[i] = D4{x, y, z, ri};
        a.vel_o[i] = D4{vx, vy, vz, mi};
        a.spin_o[i] = D4{wx, wy, wz, si.w};
    }
    if (MODE == 1) {
        if (bad) atomicOr(&a.flags->err, kErrNonFinite);
        if (need) a.flags->abort_at = step + 1;
    }
}

__global__ void k_adj_compress(AArgs a, const D4 *hin, const D4 *hwin, D4 *xi, uint64_t *mask, double *xiw) {
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int cnt = a.cnt[i];
        uint64_t m = 0;
        for (int q = 0; q < cnt; ++q) {
            const D4 h = hin[i * a.kslots + q];
            xi[i * a.kmax + q] = D4{h.x, h.y, h.z, 0.0};
            if (__double_as_longlong(h.x) | __double_as_longlong(h.y) | __double_as_longlong(h.z)) m |= 1ull << q;
        }
        const D4 hw = hwin[i];
        xiw[i] = hw.x; xiw[n + i] = hw.y; xiw[2 * n + i] = hw.z;
        if (__double_as_longlong(hw.x) | __double_as_longlong(hw.y) | __double_as_longlong(hw.z)) m |= kWallBit;
        mask[i] = m;
    }
}

__global__ void k_adj_unpack(AArgs a, double *x, double *v, double *w) {
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const D4 p = a.pos[i], u = a.vel[i], s = a.spin[i];
        x[i] = p.x; x[n + i] = p.y; x[2 * n + i] = p.z;
        v[i] = u.x; v[n + i] = u.y; v[2 * n + i] = u.z;
        w[i] = s.x; w[n + i] = s.y; w[2 * n + i] = s.z;
    }
}

// ------------------------------------------------------------ seeds

// The last evaluation of a rollout feeds the final velocities through one
// half kick: v_K = u_K + (dt/2) F / m, w_K = u_K + (dt/2) T / I.
__global__ void k_adj_seed(AArgs a, const double *gx, const double *gv, const double *gw) {
    const int64_t n = a.n;
    const double h = a.sys->hdt;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const D2 im = a.im[i];
        const double x0 = gx[i], x1 = gx[n + i], x2 = gx[2 * n + i];
        const double v0 = gv[i], v1 = gv[n + i], v2 = gv[2 * n + i];
        const double w0 = gw[i], w1 = gw[n + i], w2 = gw[2 * n + i];
        a.rout[i] = D4{x0, x1, x2, 0.0};
        a.rout[n + i] = D4{v0, v1, v2, 0.0};
        a.rout[2 * n + i] = D4{w0, w1, w2, 0.0};
        a.rout[3 * n + i] = D4{h * v0 * im.a, h * v1 * im.a, h * v2 * im.a, 0.0};
        a.rout[4 * n + i] = D4{h * w0 * im.b, h * w1 * im.b, h * w2 * im.b, 0.0};
    }
}

__global__ void k_adj_seed_forces(AArgs a, const double *fb, const double *tb) {
    const int64_t n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const D4 z = {0.0, 0.0, 0.0, 0.0};
        a.rout[i] = z;
        a.rout[n + i] = z;
        a.rout[2 * n + i] = z;
        a.rout[3 * n + i] = D4{fb[i], fb[n + i], fb[2 * n + i], 0.0};
        a.rout[4 * n + i] = D4{tb[i], tb[n + i], tb[2 * n + i], 0.0};
    }
}

// ------------------------------------------------------------ reverse

template <int NT, bool PRIME, int G>
__global__ void __launch_bounds__(kABlock, kAdjReverseWaves) k_adj_reverse(AArgs a) {
    const int64_t n = a.n;
    const int64_t ks = a.kslots;
    const SysDesc s = uniform_sys(a.sys);
    const int g = threadIdx.x % G;
    const int gbase = (threadIdx.x % warpSize) / G * G;
    const int64_t ppb = blockDim.x / G;
    const double sc = a.seed_scale;
    const bool update = !PRIME;
    for (int64_t i0 = (int64_t)blockIdx.x * ppb; i0 < n; i0 += (int64_t)gridDim.x * ppb) {
        const int64_t i = i0 + threadIdx.x / G;
        if (i >= n) continue;
        const D4 pi = a.pos[i], vi = a.vel[i], si = a.spin[i];
        const int ti = (int)si.w & 15;
        const double ri = pi.w, mi = vi.w;
        const D4 sfi = a.rin[3 * n + i], sti = a.rin[4 * n + i];
        const double Fix = sc * sfi.x, Fiy = sc * sfi.y, Fiz = sc * sfi.z;
        const double Tix = sc * sti.x, Tiy = sc * sti.y, Tiz = sc * sti.z;
        double jx0 = 0.0, jx1 = 0.0, jx2 = 0.0, ju0 = 0.0, ju1 = 0.0, ju2 = 0.0, jw0 = 0.0, jw1 = 0.0, jw2 = 0.0;
        double acc[NT][5];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int k = 0; k < 5; ++k) acc[t][k] = 0.0;
        const int cnt = a.cnt[i];
        for (int q = g; q < cnt; q += G) {
            const int64_t slot = i * ks + q;
            const int32_t j = a.nbr[q * n + i];
            const D4 pj = a.pos[j];
            ContactIn c;
            c.dx = min_image(pi.x - pj.x, s.L[0], s.hL[0], s.periodic[0]);
            c.dy = min_image(pi.y - pj.y, s.L[1], s.hL[1], s.periodic[1]);
            c.dz = min_image(pi.z - pj.z, s.L[2], s.hL[2], s.periodic[2]);
            c.ra = ri;
            c.rb = pj.w;
            const double rs = c.ra + c.rb;
            const D4 m_after = a.mu[slot];
            D4 m_before = PRIME ? m_after : D4{0.0, 0.0, 0.0, 0.0};
            if (c.dx * c.dx + c.dy * c.dy + c.dz * c.dz < rs * rs) {
                const D4 vj = a.vel[j], sj = a.spin[j];
                const D4 h = a.hin[slot];
                c.ma = mi; c.mb = vj.w;
                c.vrx = vi.x - vj.x; c.vry = vi.y - vj.y; c.vrz = vi.z - vj.z;
                c.wsx = ri * si.x + pj.w * sj.x;
                c.wsy = ri * si.y + pj.w * sj.y;
                c.wsz = ri * si.z + pj.w * sj.z;
                const int tj = (int)sj.w & 15;
                const PairCoef pc = a.coef[ti * a.ntypes + tj];
                const D4 sfj = a.rin[3 * n + j], stj = a.rin[4 * n + j];
                const double fbx = Fix - sc * sfj.x, fby = Fiy - sc * sfj.y, fbz = Fiz - sc * sfj.z;
                const double gbx = -(ri * Tix + pj.w * (sc * stj.x));
                const double gby = -(ri * Tiy + pj.w * (sc * stj.y));
                const double gbz = -(ri * Tiz + pj.w * (sc * stj.z));
                ContactAdj o;
                if (contact_vjp(c, false, pc, s.dt, update, h.x, h.y, h.z, fbx, fby, fbz, gbx, gby, gbz, m_after.x,
                                m_after.y, m_after.z, o)) {
                    jx0 += o.dbx; jx1 += o.dby; jx2 += o.dbz;
                    ju0 += o.vbx; ju1 += o.vby; ju2 += o.vbz;
                    jw0 += ri * o.wbx; jw1 += ri * o.wby; jw2 += ri * o.wbz;
                    if (PRIME) m_before = D4{m_after.x + o.xbx, m_after.y + o.xby, m_after.z + o.xbz, 0.0};
                    else m_before = D4{o.xbx, o.xby, o.xbz, 0.0};
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        if (t == tj) {
                            acc[t][0] += 0.5 * o.kn0;
                            acc[t][1] += 0.5 * o.kt0;
                            acc[t][2] += 0.5 * o.gn0;
                            acc[t][3] += 0.5 * o.gt0;
                            acc[t][4] += 0.5 * o.mu;
                        }
                }
            }
            a.mu[slot] = m_before;
        }
        if (g == 0) {
            const D4 mw_after = a.muw[i];
            D4 mw_before = PRIME ? mw_after : D4{0.0, 0.0, 0.0, 0.0};
            if (s.wall && pi.z < ri) {
                ContactIn c;
                c.dx = 0.0; c.dy = 0.0; c.dz = pi.z;
                c.ra = ri; c.rb = 0.0; c.ma = mi; c.mb = 0.0;
                c.vrx = vi.x; c.vry = vi.y; c.vrz = vi.z;
                c.wsx = ri * si.x; c.wsy = ri * si.y; c.wsz = ri * si.z;
                const PairCoef pc = a.coef[ti * a.ntypes + ti];
                const D4 h = a.hwin[i];
                ContactAdj o;
                if (contact_vjp(c, true, pc, s.dt, update, h.x, h.y, h.z, Fix, Fiy, Fiz, -(ri * Tix), -(ri * Tiy),
                                -(ri * Tiz), mw_after.x, mw_after.y, mw_after.z, o)) {
                    jx2 += o.dbz;
                    ju0 += o.vbx; ju1 += o.vby; ju2 += o.vbz;
                    jw0 += ri * o.wbx; jw1 += ri * o.wby; jw2 += ri * o.wbz;
                    if (PRIME) mw_before = D4{mw_after.x + o.xbx, mw_after.y + o.xby, mw_after.z + o.xbz, 0.0};
                    else mw_before = D4{o.xbx, o.xby, o.xbz, 0.0};
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        if (t == ti) {
                            acc[t][0] += o.kn0;
                            acc[t][1] += o.kt0;
                            acc[t][2] += o.gn0;
                            acc[t][3] += o.gt0;
                            acc[t][4] += o.mu;
                        }
                }
            }
            a.muw[i] = mw_before;
        }
        // lanes in a fixed order
        jx0 = group_sum<G>(jx0, gbase); jx1 = group_sum<G>(jx1, gbase); jx2 = group_sum<G>(jx2, gbase);
        ju0 = group_sum<G>(ju0, gbase); ju1 = group_sum<G>(ju1, gbase); ju2 = group_sum<G>(ju2, gbase);
        jw0 = group_sum<G>(jw0, gbase); jw1 = group_sum<G>(jw1, gbase); jw2 = group_sum<G>(jw2, gbase);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int k = 0; k < 5; ++k) acc[t][k] = group_sum<G>(acc[t][k], gbase);
        if (g != 0) continue;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                double *p = a.gp + (int64_t)(t * 5 + k) * n + i;
                *p = *p + acc[t][k];
            }
        const D4 ax = a.rin[i], au = a.rin[n + i], aw = a.rin[2 * n + i];
        const double xb0 = ax.x + jx0, xb1 = ax.y + jx1, xb2 = ax.z + jx2;
        const double ub0 = au.x + ju0, ub1 = au.y + ju1, ub2 = au.z + ju2;
        const double wb0 = aw.x + jw0, wb1 = aw.y + jw1, wb2 = aw.z + jw2;
        if (PRIME) {
            a.ox[i] = xb0; a.ox[n + i] = xb1; a.ox[2 * n + i] = xb2;
            a.ov[i] = ub0; a.ov[n + i] = ub1; a.ov[2 * n + i] = ub2;
            a.ow[i] = wb0; a.ow[n + i] = wb1; a.ow[2 * n + i] = wb2;
        } else {
            // x_q = x_{q-1} + dt u_q and u_q = u_{q-1} + dt F_{q-1} / m (two half kicks)
            const double dt = s.dt;
            const double p0 = ub0 + dt * xb0, p1 = ub1 + dt * xb1, p2 = ub2 + dt * xb2;
            const D2 im = a.im[i];
            a.rout[i] = D4{xb0, xb1, xb2, 0.0};
            a.rout[n + i] = D4{p0, p1, p2, 0.0};
            a.rout[2 * n + i] = D4{wb0, wb1, wb2, 0.0};
            a.rout[3 * n + i] = D4{dt * p0 * im.a, dt * p1 * im.a, dt * p2 * im.a, 0.0};
            a.rout[4 * n + i] = D4{dt * wb0 * im.b, dt * wb1 * im.b, dt * wb2 * im.b, 0.0};
        }
    }
}

// ------------------------------------------------------------ list change

__global__ void k_adj_carry(AArgs a, const int32_t *frame, const int32_t *nids, const int32_t *onbr,
                            const int32_t *ocnt, const int32_t *oids, D4 *mu_old, D4 *muw_old) {
    const int64_t n = a.n;
    const int64_t ks = a.kslots;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = frame[i];
        for (int k = 0; k < 5; ++k) a.rout[k * n + o] = a.rin[k * n + i];
        muw_old[o] = a.muw[i];
        const int cn = a.cnt[i], co = ocnt[o];
        int q = 0;
        for (int p = 0; p < co; ++p) {
            const int32_t idp = oids[onbr[p * n + o]];
            while (q < cn && nids[a.nbr[q * n + i]] < idp) ++q;
            D4 m = {0.0, 0.0, 0.0, 0.0};
            if (q < cn && nids[a.nbr[q * n + i]] == idp) m = a.mu[i * ks + q];
            mu_old[o * ks + p] = m;
        }
    }
}

// ------------------------------------------------------------ reduction

// Stage 1: block b of column col sums particles [b*chunk, (b+1)*chunk) by
// type (fixed per-thread strides, then a fixed tree) into part[col][b][type];
// stage 2: one thread per (col, type) adds the blocks in order.
constexpr int kRedBlocks = 64;

__global__ void __launch_bounds__(kABlock) k_adj_reduce1(AArgs a, double *part) {
    __shared__ double red[kMaxTypes][kABlock];
    const int col = blockIdx.y;          // tj * 5 + c
    const int64_t n = a.n;
    const int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    double p[kMaxTypes] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const int ti = (int)a.spin[i].w & 15;
        const double v = a.gp[(int64_t)col * n + i];
#pragma unroll
        for (int t = 0; t < kMaxTypes; ++t)
            if (t == ti) p[t] += v;
    }
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t) red[t][threadIdx.x] = p[t];
    __syncthreads();
    for (int w = kABlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int t = 0; t < kMaxTypes; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < kMaxTypes) part[((int64_t)col * kRedBlocks + blockIdx.x) * kMaxTypes + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_adj_reduce2(AArgs a, const double *part, double *acc) {
    const int nt = a.ntypes;
    const int k = threadIdx.x;           // col * nt + ti
    if (k >= 5 * nt * nt) return;
    const int col = k / nt, ti = k % nt;
    double s = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) s += part[((int64_t)col * kRedBlocks + b) * kMaxTypes + ti];
    const int tj = col / 5, c = col % 5;
    acc[(ti * nt + tj) * 5 + c] += s;
}

// ------------------------------------------------------------ launchers

#define CHECK_LAUNCH() return hipGetLastError()

hipError_t launch_adj_expand(const AArgs &a, const D4 *xi, const uint64_t *mask, const double *xiw, D4 *hout,
                             D4 *hwout, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    k_adj_expand<<<flat_grid(a.n), kABlock, 0, st>>>(a, xi, mask, xiw, hout, hwout);
    CHECK_LAUNCH();
}

template <int G>
static void forward_g(const AArgs &a, int mode, hipStream_t st) {
    if (mode == 1) k_adj_forward<G, 1><<<adj_grid(a.n, G), kABlock, 0, st>>>(a);
    else if (mode == 2) k_adj_forward<G, 2><<<adj_grid(a.n, G), kABlock, 0, st>>>(a);
    else k_adj_forward<G, 0><<<adj_grid(a.n, G), kABlock, 0, st>>>(a);
}

__global__ void k_adj_row_max(const int32_t *cnt, int64_t n, int32_t *out) {
    int m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, cnt[i]);
    for (int off = warpSize / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if (threadIdx.x % warpSize == 0 && m > 0) atomicMax(out, m);
}

hipError_t launch_adj_row_max(const int32_t *cnt, int64_t n, int32_t *out, hipStream_t st) {
    k_adj_row_max<<<flat_grid(n), kABlock, 0, st>>>(cnt, n, out);
    return hipGetLastError();
}

hipError_t launch_adj_forward(const AArgs &a, int mode, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    if (a.lanes == 8) forward_g<8>(a, mode, st);
    else forward_g<4>(a, mode, st);
    CHECK_LAUNCH();
}

hipError_t launch_adj_compress(const AArgs &a, const D4 *hin, const D4 *hwin, D4 *xi, uint64_t *mask, double *xiw,
                               hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    k_adj_compress<<<flat_grid(a.n), kABlock, 0, st>>>(a, hin, hwin, xi, mask, xiw);
    CHECK_LAUNCH();
}

hipError_t launch_adj_unpack(const AArgs &a, double *x, double *v, double *w, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    k_adj_unpack<<<flat_grid(a.n), kABlock, 0, st>>>(a, x, v, w);
    CHECK_LAUNCH();
}

// Reverse of one half of the velocity-Verlet step (dem_integrate), one
// thread per slot: phase 0 (kick, drift, wrap) and phase 1 (kick).  The wrap
// is a shift by a box length, so the position adjoint passes through it.
__global__ void k_integrate_vjp(const SysDesc *sys, int nsys, int64_t n, const double *inv_m, const double *inv_I,
                                int phase, const double *xb, const double *vb, const double *wb, double *xo,
                                double *vo, double *wo, double *fo, double *to) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int k = 0;
        while (k + 1 < nsys && i >= sys[k + 1].p0) ++k;
        const SysDesc &s = sys[k];
        const bool live = i >= s.p0 && i < s.pe;
        const double im = live ? inv_m[i] : 0.0, iI = live ? inv_I[i] : 0.0;
        for (int c = 0; c < 3; ++c) {
            const int64_t j = c * n + i;
            if (!live) {
                xo[j] = vo[j] = wo[j] = fo[j] = to[j] = 0.0;
                continue;
            }
            const double ux = xb[j];
            const double uv = phase == 0 ? vb[j] + s.dt * ux : vb[j];   // v' also moves x' in phase 0
            const double uw = wb[j];
            xo[j] = ux;
            vo[j] = uv;
            wo[j] = uw;
            fo[j] = s.hdt * (uv * im);
            to[j] = s.hdt * (uw * iI);
        }
    }
}

hipError_t launch_integrate_vjp(const SysDesc *sys, int nsys, int64_t n, const double *inv_m, const double *inv_I,
                                int phase, const double *xb, const double *vb, const double *wb, double *xo,
                                double *vo, double *wo, double *fo, double *to, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_integrate_vjp<<<flat_grid(n), kABlock, 0, st>>>(sys, nsys, n, inv_m, inv_I, phase, xb, vb, wb, xo, vo, wo,
                                                      fo, to);
    CHECK_LAUNCH();
}

hipError_t launch_adj_seed(const AArgs &a, const double *gx, const double *gv, const double *gw, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    k_adj_seed<<<flat_grid(a.n), kABlock, 0, st>>>(a, gx, gv, gw);
    CHECK_LAUNCH();
}

hipError_t launch_adj_seed_forces(const AArgs &a, const double *fb, const double *tb, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    k_adj_seed_forces<<<flat_grid(a.n), kABlock, 0, st>>>(a, fb, tb);
    CHECK_LAUNCH();
}

template <int NT, int G>
static void reverse_ntg(const AArgs &a, int prime, hipStream_t st) {
    if (prime) k_adj_reverse<NT, true, G><<<adj_grid(a.n, G), kABlock, 0, st>>>(a);
    else k_adj_reverse<NT, false, G><<<adj_grid(a.n, G), kABlock, 0, st>>>(a);
}

template <int NT>
static void reverse_nt(const AArgs &a, int prime, hipStream_t st) {
    if (a.lanes == 8) reverse_ntg<NT, 8>(a, prime, st);
    else reverse_ntg<NT, 4>(a, prime, st);
}

hipError_t launch_adj_reverse(const AArgs &a, int prime, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    switch (a.ntypes) {
        case 1: reverse_nt<1>(a, prime, st); break;
        case 2: reverse_nt<2>(a, prime, st); break;
        case 3: reverse_nt<3>(a, prime, st); break;
        default: reverse_nt<4>(a, prime, st); break;
    }
    CHECK_LAUNCH();
}

hipError_t launch_adj_carry(const AArgs &a, const int32_t *frame, const int32_t *nids, const int32_t *onbr,
                            const int32_t *ocnt, const int32_t *oids, D4 *mu_old, D4 *muw_old, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    k_adj_carry<<<flat_grid(a.n), kABlock, 0, st>>>(a, frame, nids, onbr, ocnt, oids, mu_old, muw_old);
    CHECK_LAUNCH();
}

size_t adj_reduce_scratch_bytes(int ntypes) { return (size_t)5 * ntypes * kRedBlocks * kMaxTypes * sizeof(double); }

hipError_t launch_adj_reduce(const AArgs &a, double *part, double *acc, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    k_adj_reduce1<<<dim3(kRedBlocks, 5 * a.ntypes), kABlock, 0, st>>>(a, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_adj_reduce2<<<1, 128, 0, st>>>(a, part, acc);
    CHECK_LAUNCH();
}

}  // namespace dem
