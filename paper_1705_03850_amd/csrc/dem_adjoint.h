// dem_adjoint.h -- kernel arguments and launchers of the reverse-mode rollout
// (internal to libdem.so).
//
// A rollout of K steps is a sequence of force evaluations at the packed states
// Y_q = (x_q, u_q, w_q) (positions, half-step velocities and spins after the
// drift of step q) with the slot history xi_{q-1}.  Evaluation q gives the
// forces, the new history xi_q and, by two half kicks and a drift, Y_{q+1}.
// The reverse pass walks the evaluations backwards.  Its per-particle adjoint
// record holds, for evaluation q - 1:
//   AX = adjoint of x_{q-1},  AU = adjoint of u_{q-1} from later use,
//   AW = adjoint of w_{q-1},  SF, ST = seeds for the force and torque of
//   evaluation q - 1 (dt AU / m and dt AW / I).
// The history adjoint is kept per slot in pair form: the adjoint of xi_ij with
// xi_ji = -xi_ij, so slot (j, i) holds the negated value of slot (i, j) and
// every particle only ever touches its own row.
#pragma once

#include "dem_core.h"

namespace dem {

struct AArgs {
    int64_t n;
    int32_t kmax;            // slots per row of the live list (its history stride)
    int32_t ntypes;
    int32_t kslots;          // slots per particle of the adjoint's own history buffers (<= kmax)
    int32_t pad_a;
    const SysDesc *sys;      // the system
    const PairCoef *coef;    // ntypes x ntypes
    // topology of the window (order of its list build)
    const int32_t *nbr, *cnt;
    const D2 *im;            // (1/m, 1/I)
    // the evaluation's input state
    const D4 *pos, *vel, *spin;
    const D4 *hin;           // [n][kslots] slot history before the evaluation, zero where none
    const D4 *hwin;          // [n] wall history before the evaluation
    // recompute outputs
    D4 *pos_o, *vel_o, *spin_o, *hout, *hwout;
    // reverse
    const D4 *rin;           // [5][n] adjoint records (AX, AU, AW, SF, ST)
    D4 *rout;
    D4 *mu;                  // [n][kslots] slot history adjoint (in: after, out: before the evaluation)
    D4 *muw;                 // [n] wall history adjoint
    double *gp;              // [5 ntypes][n] coefficient adjoint partials of each particle
    double seed_scale;       // factor on the seeds read from rin
    int32_t lanes;           // threads per particle in the recompute and reverse passes (4 or 8)
    double *ox, *ov, *ow;    // priming evaluation: adjoints of the initial x, v, w ([3][n])
    // the forward of a kept rollout (forward modes 1 and 2)
    Flags *flags;            // gating: this evaluation is step step_base + k
    int32_t k;
    double *disp;            // [3][n] displacement since the last list build
    double *x, *v, *w, *f, *t;   // caller arrays, written by the last step
};

// Live list (ELL rows with the non-zero-history mask) -> full-form history.
hipError_t launch_adj_expand(const AArgs &a, const D4 *xi, const uint64_t *mask, const double *xiw, D4 *hout,
                             D4 *hwout, hipStream_t st);
// One evaluation: pos/vel/spin, hin, hwin -> *_o, hout, hwout, with the arithmetic
// and summation order of the fused step.  mode 0: recompute; mode 1: a step of
// a kept rollout (gated like the fused step; displacement, rebuild request and
// non-finite check); mode 2: its last step (gated; forces, one half kick, and
// x, v, w, f, t written to the caller's arrays; no drift).
hipError_t launch_adj_forward(const AArgs &a, int mode, hipStream_t st);
// Full-form history -> live list rows (history and mask; mask bit where the
// stored value is not all zero bits) and wall history [3][n].
hipError_t launch_adj_compress(const AArgs &a, const D4 *hin, const D4 *hwin, D4 *xi, uint64_t *mask, double *xiw,
                               hipStream_t st);
// Longest row of a list (cnt[n]) -> atomic maximum into *out (cleared by the caller).
hipError_t launch_adj_row_max(const int32_t *cnt, int64_t n, int32_t *out, hipStream_t st);
// Reverse of dem_integrate's phase 0 or 1: output adjoints (xb, vb, wb) ->
// input adjoints (xo, vo, wo) and force and torque adjoints (fo, to), [3][n].
hipError_t launch_integrate_vjp(const SysDesc *sys, int nsys, int64_t n, const double *inv_m, const double *inv_I,
                                int phase, const double *xb, const double *vb, const double *wb, double *xo,
                                double *vo, double *wo, double *fo, double *to, hipStream_t st);
// Packed pos/vel/spin -> caller arrays x, v, w.
hipError_t launch_adj_unpack(const AArgs &a, double *x, double *v, double *w, hipStream_t st);
// Records of the last evaluation from the adjoints of the final x, v, w.
hipError_t launch_adj_seed(const AArgs &a, const double *gx, const double *gv, const double *gw, hipStream_t st);
// Records for the reverse of a single force evaluation (seeds = force and torque adjoints).
hipError_t launch_adj_seed_forces(const AArgs &a, const double *fb, const double *tb, hipStream_t st);
// Reverse of one evaluation: prime = 0 for a step (history updated), 1 for
// the first force evaluation of a rollout (history untouched; writes ox, ov, ow).
hipError_t launch_adj_reverse(const AArgs &a, int prime, hipStream_t st);
// Across a list rebuild: records and wall adjoint permuted to the previous
// order (frame: new index -> previous index), slot adjoints matched by id.
hipError_t launch_adj_carry(const AArgs &a, const int32_t *frame, const int32_t *nids, const int32_t *onbr,
                            const int32_t *ocnt, const int32_t *oids, D4 *mu_old, D4 *muw_old, hipStream_t st);
// acc[(ti ntypes + tj) 5 + c] += sum over particles of type ti of gp[(tj 5 + c)][i], in a
// fixed order; part is scratch of adj_reduce_scratch_bytes(ntypes).
hipError_t launch_adj_reduce(const AArgs &a, double *part, double *acc, hipStream_t st);
size_t adj_reduce_scratch_bytes(int ntypes);

}  // namespace dem
