// dem_kernels.h -- kernel arguments and launchers of libdem.so (internal).
#pragma once

#include "dem_core.h"

namespace dem {

// doubles per particle in the binning scratch: x, v, w, f, t, disp, wall history,
// external force (3 each), r, m, 1/m, 1/I
constexpr int kShadowD = 28;

// strides of multi-rate stepping: 1, 2, 4, ..., 2^(kMaxLevels - 1)
constexpr int kMaxLevels = 11;

// Everything a kernel may touch, passed by value.
struct KArgs {
    // caller-owned particle arrays
    double *x, *v, *w, *f, *t, *r;
    int32_t *type, *id;
    // library-owned per-particle arrays (workspace)
    double *m, *inv_m, *inv_I, *disp, *xiw;
    int32_t *frame;        // index of each particle in the order of the last list build (-1: none)
    int32_t *dead;         // [n] 1 = removed at the next binning of its system (insertion events)
    double *fext_ws;       // [3][n] external forces (workspace)
    const double *fext;    // fext_ws while external forces are on, else null
    // static wall surfaces (null when no system has any)
    const Surf *surf;      // [nsys * kMaxSurf]
    D4 *sxi;               // [nsurf_slots][n] tangential history of each surface contact
    uint32_t *smask;       // [n] bit k: surface k holds non-zero history
    double *shadow_s;      // binning scratch of sxi ([3 nsurf_slots][n] doubles) then smask ([n] words)
    int32_t nsurf_slots;
    int32_t pad_s;
    // systems
    const SysDesc *sys;
    const PairCoef *coef;
    const double *rho;     // per type, all systems
    int32_t nsys;
    int32_t kmax;
    int32_t block;
    int32_t grid_cap;      // blocks of the fused step kernel (0 = one per tile)
    int32_t lanes;         // lanes per particle in the force pass: 4, 8 or 16
    int32_t multirate;     // systems step every SysDesc::stride substeps (batch only)
    int64_t n;             // particles, all systems
    int64_t ncell;         // cells, all systems
    // window of the rebuild kernels (particles [w0, w1), cells [cw0, cw1)): the
    // index ranges of the systems selected for a rebuild; everything otherwise
    int64_t w0, w1, cw0, cw1;
    int64_t call_steps;    // set only for the last step of a dem_step call: added to the step count
    int32_t only_sys;      // >= 0: the force pass of one system only (the others' f, t kept); -1: all
    int32_t pad_k;
    Flags *flags;
    List lst[2];           // two list buffers; system s uses lst[lcur[s]], builds into the other
    int32_t *lcur;         // [nsys] current list buffer of each system
    // binning scratch
    int32_t *cell_of, *rank, *cell_count, *cell_start, *scan_partial, *order;
    double *shadow_d;      // [kShadowD][n]
    int32_t *shadow_i;     // [3][n]
    // packed step state, two buffers used alternately
    D4 *pos[2], *vel[2], *spin[2];
    D2 *im;                // (1/m, 1/I)
    int32_t *sel;          // [nsys] 1 = system needs (or gets) a new list
    // batch step: tiles of block / lanes particles, each within one system;
    // system s has tiles tile0[s] .. tile0[s+1]-1
    const int64_t *tile0;  // [nsys + 1]
    int64_t ntiles_b;
    // multi-rate: the same tiles with the systems ordered by stride (msys[k] is the
    // k-th system, its tiles mtile0[k] .. mtile0[k+1]-1), so that the tiles of the
    // systems stepping at a substep form the prefix [0, mlevel[l]) for the largest
    // l with 2^l dividing the substep's index
    const int64_t *mtile0; // [nsys + 1]
    const int32_t *msys;   // [nsys]
    const int64_t *mlevel; // [kMaxLevels]
};

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t st);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t st);
hipError_t launch_ctrl(Flags *f, int op, int64_t value, hipStream_t st);
hipError_t launch_init_mass(const KArgs &a, hipStream_t st);
hipError_t launch_phase(const KArgs &a, int phase, int k, int gate, hipStream_t st);
// exclusive scan of in[0..m) into out[0..m] (out[m] = total); partial holds
// (m + 1023) / 1024 + 1 words
hipError_t launch_scan(const int32_t *in, int64_t m, int32_t *partial, int32_t *out, hipStream_t st);
hipError_t launch_bin(const KArgs &a, int frame_identity, hipStream_t st);
hipError_t launch_neighbors(const KArgs &a, int have_old, hipStream_t st);
// after a build: the selected systems switch to their new list buffer
hipError_t launch_flip(const KArgs &a, hipStream_t st);
// mode 0: pack only; 1: pack and do phase 0 of step `k` (gated); 2: pack the
// particles of the systems selected for a rebuild only (in multi-rate mode into
// each system's buffer for substep qa of the call, qa >= 1)
hipError_t launch_pack(const KArgs &a, int dst, int mode, int k, int gate, hipStream_t st, int64_t qa = 0);
// selected != 0: only particles of systems selected for a rebuild (multi-rate:
// from each system's buffer for substep qa of the call)
hipError_t launch_unpack(const KArgs &a, int src, int selected, hipStream_t st, int64_t qa = 0);
// force pass over packed buffer src: mode 0 forces only (to f, t); mode 1 fused
// step (forces, kick, next kick + drift into buffer src^1); mode 2 last step
// (forces, kick, f, t, x, v, w to the caller's arrays).
hipError_t launch_step(const KArgs &a, int src, int mode, int k, int update, int count, hipStream_t st);

}  // namespace dem
