/*
 * dem.h -- C-ABI of libdem.so, the MI355X (gfx950) DEM contact pipeline.
 *
 * One call of dem_step advances soft spheres by velocity Verlet under the
 * contact law of Queteschiner et al., "Adaptive Coarse-Graining for
 * Large-Scale DEM Simulations" (CFD2017):
 *   Newton's equations for translation and rotation ............ Sec. 2.1, Eq. (1)-(2)
 *   force = gravity + binary contact forces ..................... Sec. 2.1
 *   damped Hertz normal force .................................... Eq. (3), Eq. (6)
 *   tangential spring-dashpot with overlap history ............... Eq. (4), Eq. (6)
 *   Coulomb truncation f_t <= mu f_n ............................. Eq. (5)
 *   coarse-grain rule (E, nu, rho, e, mu fixed, radius scaled) .... Sec. 2.2
 *   several coarse-grain levels as one batch of systems ........... Sec. 2.3
 * The readings where the paper is silent (effective properties, sign
 * conventions, history rules, the integrator) are the same as the CPU
 * oracle's and are listed in the repository's design notes.
 *
 * Conventions
 *   - Units are SI.  All floating point is IEEE binary64.
 *   - Particle arrays are device memory owned by the caller, structure of
 *     arrays: a vector field V of n particles is V[0..n) = x components,
 *     V[n..2n) = y, V[2n..3n) = z.
 *   - A batch of S systems concatenates the systems' particle slots: system s
 *     owns the index range [off_s, off_s + m_s), m_s = dem_config.n_max (n when
 *     0), with off_0 = 0 in the order of the configurations passed to
 *     dem_batch_init.  Its live particles are the first slots of that range,
 *     [off_s, off_s + live_s): n of them at first; dem_exchange changes the
 *     count (dem_live_count reads it).  Slots past the live ones are ignored
 *     by every call.  Every call below acts on all systems of the context.
 *   - Ids must be unique across the whole context (all systems of a batch)
 *     and non-negative.  dem_bin permutes the caller's particle arrays (within
 *     each system); compare results by id.
 *   - The library never allocates device memory.  Its device storage is one
 *     caller-provided workspace of dem_workspace_size() bytes that must stay
 *     allocated and untouched until dem_destroy.  dem_init and dem_batch_init
 *     allocate one small pinned host buffer (the copy of the flag block that
 *     synchronising calls read), freed by dem_destroy; dem_init_noalloc
 *     allocates nothing.
 *   - Calls are enqueued on the stream given to dem_init (a hipStream_t passed
 *     as void*) and return before the GPU finishes, except where a call is
 *     documented as synchronising.
 *   - Every call returns DEM_OK or a DEM_ERR_* code; nothing aborts or throws
 *     across this boundary.  dem_last_error() gives a message for the last
 *     failing call on a context.  Errors found by kernels (list capacity,
 *     non-finite values) are sticky device flags that dem_check, dem_step and
 *     the export calls report.
 */
#ifndef DEM_H
#define DEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DEM_OK = 0,
    DEM_ERR_ARG = 1,        /* invalid argument or configuration              */
    DEM_ERR_CAPACITY = 2,   /* a neighbour row needs more than k_max slots    */
    DEM_ERR_DOMAIN = 3,     /* box too small for the cut-off, or bad geometry */
    DEM_ERR_NONFINITE = 4,  /* NaN or infinity in positions or velocities      */
    DEM_ERR_HIP = 5,        /* a HIP runtime call failed                       */
    DEM_ERR_STATE = 6       /* call out of order (e.g. forces before a list)   */
};

#define DEM_MAX_TYPES 4
#define DEM_MAX_SURFACES 4

/* Material of one particle type (Sec. 2.1 and Sec. 2.2).  A pair of two
 * types uses the harmonic effective modulus and shear modulus of the two
 * materials, e = (e_i + e_j)/2 and mu = (mu_i + mu_j)/2; the flat wall is
 * treated as the contacting particle's own material. */
typedef struct dem_material {
    double E;    /* Young's modulus (Pa), > 0                 */
    double nu;   /* Poisson ratio, in (-1, 0.5)               */
    double rho;  /* density (kg/m^3), > 0                     */
    double e;    /* coefficient of restitution, in (0, 1]     */
    double mu;   /* Coulomb friction coefficient, >= 0        */
} dem_material;

/* One system.  The box [lo, hi) is the periodic cell along periodic axes and
 * the extent of the binning grid along open axes (particles outside an open
 * axis are still handled correctly, they share the edge cells). */
typedef struct dem_config {
    int32_t ntypes;                    /* 1..DEM_MAX_TYPES                              */
    dem_material mat[DEM_MAX_TYPES];
    double dt;                         /* time step (s), > 0                            */
    double g[3];                       /* gravity (m/s^2)                               */
    double lo[3], hi[3];               /* box corners (m), hi > lo                      */
    int32_t periodic[3];               /* 1 = periodic axis                              */
    int32_t wall_z0;                   /* 1 = flat frictional wall at z = 0, normal +z  */
    double skin;                       /* neighbour-list skin s (m), > 0                */
    double cell;                       /* cell edge (m); 0 = smallest valid, 2 r_max + s */
    double r_max;                      /* largest particle radius in this system (m)    */
    int64_t n;                         /* particle count, >= 0                          */
    int32_t k_max;                     /* neighbour slots per particle, 1..63           */
    int32_t block;                     /* threads per block: 64, 128, 256; 0 = 256      */
    int64_t n_max;                     /* particle slots, >= n (room for insertion);
                                          0 = n                                          */
    int32_t n_surf;                    /* static wall surfaces reserved, 0..DEM_MAX_SURFACES
                                          (dem_set_surfaces)                             */
    int32_t pad;
} dem_config;

/* Caller-owned device arrays of the particles (see Conventions). */
typedef struct dem_state {
    double *x;       /* [3][n] positions (m); kept wrapped into [lo, hi) on periodic axes */
    double *v;       /* [3][n] velocities (m/s)                                        */
    double *w;       /* [3][n] angular velocities (rad/s)                              */
    double *f;       /* [3][n] force of the last force evaluation (N)                  */
    double *t;       /* [3][n] torque of the last force evaluation (N m)               */
    double *r;       /* [n] radius (m)                                                 */
    int32_t *type;   /* [n] material index into dem_config.mat                         */
    int32_t *id;     /* [n] particle id, unique within the context, >= 0                */
} dem_state;

typedef struct dem_ctx dem_ctx;

/* Device workspace bytes for one system (host only, no device work). */
int dem_workspace_size(const dem_config *cfg, size_t *bytes);

/* Same for a batch of nsys systems (Sec. 2.3: levels of different coarse-grain
 * factor as independent systems of one launch). */
int dem_batch_workspace_size(int32_t nsys, const dem_config *cfgs, size_t *bytes);

/* Create a context over a caller-owned device workspace (at least the size
 * returned above, 256-byte aligned).  stream: hipStream_t as void* (NULL =
 * the default stream).  Validates the configuration: DEM_ERR_ARG for bad
 * materials, dt, skin, k_max or block, DEM_ERR_DOMAIN when a periodic box is
 * shorter than two cut-offs (2 (2 r_max + skin)).  Synchronises once. */
int dem_init(dem_ctx **ctx, const dem_config *cfg, void *workspace, size_t ws_bytes, void *stream);
int dem_batch_init(dem_ctx **ctx, int32_t nsys, const dem_config *cfgs, void *workspace, size_t ws_bytes,
                   void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): dem_init of one
 * system with the workspace placed in the library's static device array of
 * 64 MiB (67,108,864 bytes) instead of a caller buffer.  Each device holds
 * its own array from the library's load to the end of the process; this call
 * takes its address for the current device, clears the part the system needs
 * (the array keeps the previous context's contents) and calls no allocating
 * routine for device memory (the context itself is host memory, as with
 * dem_init).  Only one context per device may use the array at a time:
 * DEM_ERR_STATE while another lives (dem_destroy releases it, after
 * synchronising its stream).  Work of two such contexts on one device must
 * not overlap in time; it would race on the array.  DEM_ERR_CAPACITY (before
 * any device work) when dem_workspace_size(cfg) exceeds the array, e.g. beyond
 * about 20,000 particles at k_max = 32; other errors as dem_init.  The
 * context is used and destroyed like any other. */
int dem_init_noalloc(dem_ctx **ctx, const dem_config *cfg, void *stream);

/* Start from the particles in *s: computes masses m = (4/3) pi rho r^3 and
 * inertias I = (2/5) m r^2 (solid spheres, Eq. (1)-(2)), clears the tangential
 * history of all pairs and of the wall, and marks the neighbour list invalid.
 * Synchronises; DEM_ERR_ARG when a type is out of range, an id negative or a
 * radius not positive. */
int dem_reset(dem_ctx *ctx, const dem_state *s);

/* Binning: sorts every system's particles by cell (cell index major, id minor)
 * with a counting sort and permutes all caller arrays and the library's
 * per-particle data in place.  The stored history is kept and re-attached to
 * the particles by the next dem_neighbors. */
int dem_bin(dem_ctx *ctx, const dem_state *s);

/* Neighbour list: for every particle i all j with d^2 < (r_i + r_j + skin)^2
 * (minimum image), one row per particle sorted by neighbour id.  The
 * tangential history of every pair still listed is carried over from the
 * previous list by id; new pairs start with zero history.  Requires dem_bin
 * on the current positions (DEM_ERR_STATE otherwise). */
int dem_neighbors(dem_ctx *ctx, const dem_state *s);

/* Force and torque on every particle (Eq. (3)-(6), gravity, the wall) at the
 * current positions and velocities, written to s->f and s->t.  With
 * update_history != 0 the tangential overlaps are advanced by v_t dt and
 * truncated (Eq. (5)) and stored; with 0 they are only read (the first force
 * evaluation of a run).  Uses no atomics: each particle sums its own row
 * (gravity, then neighbours by ascending id, then the wall), so results do
 * not depend on the particle order.  Requires a list (DEM_ERR_STATE). */
int dem_forces(dem_ctx *ctx, const dem_state *s, int update_history);

/* Velocity Verlet halves.  phase 0: v += dt/2 f/m, w += dt/2 t/I, x += dt v,
 * wrap periodic axes, accumulate the displacement since the last list build.
 * phase 1: v += dt/2 f/m, w += dt/2 t/I.  DEM_ERR_ARG for another phase. */
int dem_integrate(dem_ctx *ctx, const dem_state *s, int phase);

/* nsteps velocity-Verlet steps: phase 0, rebuild (bin + list) when some
 * particle moved more than skin/2 since the last build, forces with history
 * update, phase 1.  The step loop runs on a packed copy of the particles in
 * the workspace, with one fused kernel per step (forces, kick, and the next
 * step's kick and drift); the caller's arrays are read at the start and
 * written at the end.  Results are bit-identical to calling dem_integrate(0),
 * dem_bin/dem_neighbors when needed, dem_forces(1) and dem_integrate(1).
 * The first half kick of velocity Verlet uses s->f and s->t, so they must be
 * the forces of the current state: the context tracks this and returns
 * DEM_ERR_STATE (stepping nothing) unless, since the last dem_reset,
 * dem_set_materials or dem_integrate(ctx, s, 0), the forces were evaluated
 * (dem_forces, a previous dem_step or dem_rollout_forward) or declared with
 * dem_declare_forces.  dem_bin and dem_neighbors keep them valid (they permute
 * f and t with the particles).  The rebuild decision is taken on the device;
 * the host learns of it at a synchronisation every few dozen steps, so this
 * call synchronises the stream.  Returns the sticky device errors
 * (DEM_ERR_CAPACITY, DEM_ERR_NONFINITE). */
int dem_step(dem_ctx *ctx, const dem_state *s, int64_t nsteps);

/* The caller states that s->f and s->t hold the force and torque of the
 * current positions and velocities (restored from a checkpoint, computed
 * elsewhere), so that dem_step may take its first half kick from them
 * (velocity Verlet, Eq. (1)-(2)).  Host only; nothing is checked on the
 * device. */
int dem_declare_forces(dem_ctx *ctx);

/* Multi-rate stepping of a batch (Sec. 2.3: coarse-grain levels nested
 * recursively; Sec. 3: the time step may grow with the coarse-grain factor).
 * With enable != 0 every system s steps with its own dt_s once every
 * stride_s = dt_s / dt_min substeps, so that all systems reach the same time
 * at the end of every largest stride; nsteps of dem_step then counts substeps
 * of dt_min and must be a multiple of the largest stride (DEM_ERR_ARG).  Every
 * dt_s must be dt_min times a power of two up to 1024 (DEM_ERR_ARG).  Each
 * system's trajectory is bit for bit the one it has stepped alone with its dt
 * for nsteps / stride_s steps.  A single system needs no strides (ignored).
 * enable == 0 returns to one step per system per substep.  Synchronises. */
int dem_set_multirate(dem_ctx *ctx, int enable);

/* Step-loop options: use_graph != 0 replays the per-step kernels as one
 * captured HIP graph of `chunk` steps (chunk even, 2..1024; default 64). */
int dem_set_step_options(dem_ctx *ctx, int use_graph, int32_t chunk);

/* Per-kernel timing for measurement.  With enable != 0, dem_step launches
 * its kernels one by one (no graph replay) and brackets them with pairs of
 * HIP events on the context's stream: one pair around each run of fused
 * steps between synchronisations, one around each other launch (events are
 * created on first use and released by dem_destroy); enabling or disabling
 * clears the totals. */
int dem_set_timing(dem_ctx *ctx, int enable);

/* Accumulated GPU time (ms) and launch count of each timed kernel class of
 * dem_step since timing was enabled: [0] the first kick-drift of a call
 * (with packing of the caller arrays), [1] the fused step (forces, kick,
 * next kick-drift), [2] the last step of a call (forces, kick, write-back),
 * [3] list rebuild (unpack, bin, neighbours, repack).  Synchronises. */
int dem_kernel_times(dem_ctx *ctx, double ms[4], int64_t launches[4]);

/* Launch shape of the force pass: `lanes` threads per particle (4, 8 or 16; a
 * particle's row is split over them; 0 = the default, also set at init: the
 * most of 4, 8 and 16 with n * lanes <= 65536, else 4) and at most max_blocks
 * workgroups, each walking several tiles of particles (0 = as many as stay
 * resident on the device).  The schedule changes, the results do not: the
 * pair terms of a row are always added in neighbour-id order.  In a batch
 * every tile of particles lies within one system; the per-system tile table
 * for the new shape is uploaded here.  Synchronises. */
int dem_set_launch(dem_ctx *ctx, int32_t lanes, int32_t max_blocks);

/* Synchronise and report the sticky device flags.  info[0] = error bits
 * (1 capacity, 2 non-finite), info[1] = largest neighbour row seen (the k_max
 * a retry needs), info[2] = list builds so far, info[3] = steps so far.
 * Returns DEM_ERR_CAPACITY / DEM_ERR_NONFINITE when flagged. */
int dem_check(dem_ctx *ctx, int64_t info[4]);

/* Counters (synchronises): out[0] steps, out[1] list builds, out[2] sum over
 * force evaluations of directed contacts (each unordered pair counts twice),
 * out[3] sum of wall contacts, out[4] listed directed slots of the current
 * list. */
int dem_stats(dem_ctx *ctx, int64_t out[5]);

/* Host copies for checking (synchronise).  Output arrays are host memory of
 * `cap` entries; *count receives the total even when it exceeds cap.
 *   dem_export_neighbors: directed list entries (id_i, id_j), sorted.
 *   dem_export_contacts:  directed pairs in contact at the current positions
 *                         with their tangential history xi_ij [count][3].
 *   dem_export_wall:      particles touching the wall and their history. */
int dem_export_neighbors(dem_ctx *ctx, const dem_state *s, int32_t *id_i, int32_t *id_j, int64_t cap,
                         int64_t *count);
int dem_export_contacts(dem_ctx *ctx, const dem_state *s, int32_t *id_i, int32_t *id_j, double *xi, int64_t cap,
                        int64_t *count);
int dem_export_wall(dem_ctx *ctx, const dem_state *s, int32_t *id, double *xi, int64_t cap, int64_t *count);

/* Set the tangential history from host arrays (synchronises): npairs directed
 * entries (id_i, id_j, xi[3]) and nwall wall entries (id, xi[3]).  Pairs in the
 * current list that are not given get zero history.  Requires a list
 * (DEM_ERR_STATE). */
int dem_import_history(dem_ctx *ctx, const dem_state *s, int64_t npairs, const int32_t *id_i, const int32_t *id_j,
                       const double *xi, int64_t nwall, const int32_t *wall_id, const double *wall_xi);

/* ---------------------------------------------------------------------------
 * Coupling of coarse-grain levels (Sec. 2.3).
 *
 * A fine region is embedded in a coarse-grain simulation; both are systems
 * (of one batch or of two contexts).  Per hexahedral cell the library reduces
 * the Eulerian fields of a system (the granular stress of Eq. (7), the volume
 * fraction, the Favre-averaged and the maximum velocity).  Two controllers turn
 * the fields of the two levels into correcting forces: a PI controller on the
 * fine spheres of the transition layer (fine normal stress towards the coarse
 * one, force limited by the coarse maximum velocity, fading out 3/2 fine
 * diameters from the boundary) and a P controller on the coarse spheres inside
 * the fine region (velocity or mass flow).  The forces are external forces:
 * every later force evaluation adds them after the wall term, until they are
 * replaced or cleared.  The readings where the paper is silent (cell
 * membership by centre, the force's distribution over spheres, the gains) are
 * listed in the repository's design notes.
 * ------------------------------------------------------------------------- */

/* A regular grid of cells in one system's coordinates.  A sphere belongs to
 * the cell that contains its centre: c_a = floor((x_a - lo_a) / h_a), inside
 * when 0 <= c_a < n_a on every axis.  Cell (a, b, c) has index
 * (c n[1] + b) n[0] + a.  On periodic axes the cells should lie within the
 * system's box [lo, hi) (positions are kept there). */
typedef struct dem_grid {
    double lo[3];     /* corner of cell (0, 0, 0) (m)                  */
    double h[3];      /* cell edges (m), > 0                           */
    int32_t n[3];     /* cells per axis, >= 1 (at most 2^24 cells)     */
    int32_t sys;      /* system of the context whose spheres are used  */
} dem_grid;

/* Rows of a fields array: device doubles [DEM_NFIELDS][ncell] (row major, a
 * row per quantity, ncell = n[0] n[1] n[2]). */
enum {
    DEM_F_COUNT = 0,    /* spheres in the cell                                            */
    DEM_F_MASS = 1,     /* sum of m                                                        */
    DEM_F_MOM = 2,      /* rows 2..4: sum of m v (x, y, z); Favre velocity = MOM / MASS    */
    DEM_F_VOLUME = 5,   /* sum of (4/3) pi r^3; volume fraction = VOLUME / cell volume     */
    DEM_F_VMAX = 6,     /* max |v|                                                         */
    DEM_F_STRESS = 7,   /* rows 7..15: sigma_ab of Eq. (7), row 7 + 3 a + b (Pa)           */
    DEM_NFIELDS = 16
};

/* Cell fields of the system grid->sys at the current state (Sec. 2.3, Eq. (7)):
 * sigma = (1/V) sum over the cell's spheres i of [sum over contacts j of
 * 1/2 d_ij f_ij^T + m_i v'_i v'_i^T], V the cell volume, d_ij = x_i - x_j
 * (minimum image), f_ij the contact force on i at the current positions,
 * velocities and stored history (a force evaluation without history update;
 * wall contacts do not enter), v' = v - u with u the cell's Favre velocity.
 * Sums run in a fixed order (reproducible results).  Needs the neighbour list
 * of the current order (DEM_ERR_STATE) and spheres within one list cell of the
 * positions of the last list build (the state after dem_step always is): a
 * sphere found farther sets a sticky device error that the next synchronising
 * call (dem_check, dem_step, dem_exchange) reports as DEM_ERR_STATE, and the
 * controllers then leave the external forces as they are.  fields: device,
 * caller-owned.  Enqueued (no synchronisation). */
int dem_cell_fields(dem_ctx *ctx, const dem_state *s, const dem_grid *grid, double *fields);

/* The same without the stress: rows DEM_F_COUNT to DEM_F_VMAX as above, bit
 * for bit; the stress rows of fields are not written.  Enough for the P
 * controller and for an insertion budget (Sec. 2.3), which read only mass,
 * momentum and volume.  Same requirements, errors and ordering. */
int dem_cell_mass_fields(dem_ctx *ctx, const dem_state *s, const dem_grid *grid, double *fields);

/* PI controller of the transition layer (Sec. 2.3).  grid: the transition
 * cells, in the fine system grid.sys.  fine, coarse: fields (as above) of the
 * fine system and of the coarse system on the same cells.  Per cell, with the
 * unit normal nrm pointing into the fine region: e = nrm.sigma_c.nrm -
 * nrm.sigma_f.nrm, integral += e interval, u = kp e + ki integral; integral
 * (device [ncell], caller state, in/out) and u (device [ncell], out).  Then
 * every sphere of the fine system gets the external force
 * u pi r^2 w nrm in a transition cell, 0 elsewhere, where w = 1 - s/(fade 2 r)
 * for depth s = x.nrm - face in [0, fade 2 r) (1 above the face, 0 below
 * that depth), limited so that a sphere's velocity along nrm does not pass
 * the coarse cell's maximum velocity after one step (and never reversed).
 * External forces of other systems are kept. */
typedef struct dem_pi_params {
    dem_grid grid;
    double nrm[3];      /* unit normal into the fine region                        */
    double face;        /* boundary face: the plane x . nrm = face                 */
    double kp, ki;      /* gains: u = kp e + ki integral (kp: 1, ki: 1/s)          */
    double interval;    /* coupling interval (s) added to the integral per call    */
    double fade;        /* fade-out depth in fine diameters (the paper's 3/2)      */
} dem_pi_params;
int dem_pi_control(dem_ctx *ctx, const dem_state *s, const dem_pi_params *p, const double *fine,
                   const double *coarse, double *integral, double *u);

/* P controller of the coarse system grid.sys inside the fine region (Sec.
 * 2.3).  fine, coarse: fields of the two systems on the same cells.  Where both
 * cells hold mass: target = u_f (velocity) or u_f phi_f / phi_c (mass flow,
 * the fine velocity times the volume-fraction mismatch), and every coarse
 * sphere of the cell gets the external force kp m (target - u_c); the others
 * of the system get 0.  External forces of other systems are kept. */
typedef struct dem_p_params {
    dem_grid grid;
    double kp;          /* gain (1/s)                                  */
    int32_t mass_flow;  /* 0: velocity, 1: mass flow                    */
} dem_p_params;
int dem_p_control(dem_ctx *ctx, const dem_state *s, const dem_p_params *p, const double *fine,
                  const double *coarse);

/* Coupled stepping: nintervals coupling intervals of the multi-level model
 * (Sec. 2.3: fields, PI and P controllers every interval_steps steps), each
 * bit for bit the same as the calls
 *   dem_cell_fields(pi.grid -> pi_fine);
 *   dem_cell_fields(pi.grid with sys = pi_setpoint_sys -> pi_coarse);
 *   dem_pi_control(pi, pi_fine, pi_coarse, integral, u);
 *   dem_cell_mass_fields(p.grid with sys = p_target_sys -> p_fine);
 *   dem_cell_mass_fields(p.grid -> p_coarse);
 *   dem_p_control(p, p_fine, p_coarse);
 *   if sum: dem_cell_mass_fields(sum_grid -> sum_tmp), then sum += sum_tmp;
 *   dem_step(interval_steps);
 * but with one synchronisation per `group` intervals instead of one per
 * interval: the intervals of a group are enqueued together, a drift that asks
 * for a list rebuild stops every later kernel of the group (the coupling
 * kernels and steps skip their work while a rebuild is pending), and the call
 * rebuilds, finishes the interrupted interval and issues the skipped
 * intervals again.  Field arrays: device, DEM_NFIELDS rows of the grid's
 * cells (the stress rows of p_fine, p_coarse and sum_tmp are not written).
 * Same requirements and errors as those calls (DEM_ERR_STATE without the
 * forces of the current state, DEM_ERR_ARG for a bad plan; with multi-rate
 * stepping interval_steps must be a multiple of the largest stride).
 * Synchronises once per group. */
typedef struct dem_coupling_plan {
    dem_pi_params pi;          /* PI controller; pi.grid: transition cells of the fine system    */
    int32_t pi_setpoint_sys;   /* coarse system whose fields on pi.grid's cells are the setpoint */
    int32_t p_target_sys;      /* fine system whose fields on p.grid's cells are the target      */
    dem_p_params p;            /* P controller; p.grid: cells of the coarse system               */
    double *pi_fine, *pi_coarse, *p_fine, *p_coarse;   /* fields written every interval      */
    double *integral, *u;      /* PI state (in/out) and output, [cells of pi.grid]                */
    dem_grid sum_grid;         /* cells whose fields (without stress) are summed every interval   */
    double *sum, *sum_tmp;     /* running sum (in/out) and scratch; sum NULL: no summing          */
    int64_t interval_steps;    /* steps per interval, >= 1                                        */
    int32_t group;             /* intervals per synchronisation, >= 1                             */
    int32_t pad;
} dem_coupling_plan;
int dem_step_coupled(dem_ctx *ctx, const dem_state *s, int64_t nintervals, const dem_coupling_plan *plan);

/* Set the external forces of all spheres from a device array [3][n] in the
 * current order (copied), or clear them (fext NULL).  They are added to every
 * later force evaluation (after gravity, the contacts and the wall) and move
 * with the spheres when dem_bin reorders them.  The reverse mode refuses
 * contexts with external forces (DEM_ERR_STATE). */
int dem_set_external_force(dem_ctx *ctx, const dem_state *s, const double *fext);

/* ---------------------------------------------------------------------------
 * Static wall surfaces (the silo of Sec. 3: a cylinder on a cone, closed by a
 * plug over the orifice that is removed to start the discharge).
 *
 * Up to dem_config.n_surf surfaces per system, each around the vertical axis
 * through (axis[0], axis[1]).  A surface is a wall of the touching particle's
 * own material, like the flat wall, seen as flat at the contact point: the
 * contact point is the nearest point of the surface to the centre, the normal
 * the unit vector from it to the centre and the overlap r - d for a centre at
 * distance 0 < d < r on the inner side; each surface keeps its own tangential
 * history per particle.  The force pass adds a particle's surface terms after
 * its flat-wall term, in table order.  Kinds:
 *   DEM_SURF_CYLINDER  inside of radius r0 for z0 <= z <= z1 (centre's height);
 *   DEM_SURF_CONE      inside of the frustum of radius r0 at z0 and r1 at z1
 *                      (the foot of the centre's perpendicular on the slanted
 *                      side within it);
 *   DEM_SURF_DISK      the disk of radius r0 at height z0, touched from above
 *                      by centres within r0 of the axis;
 *   DEM_SURF_RING      the circle of radius r0 at height z0 (an edge).
 * A centre on or behind a surface, or on the axis of a cylinder, cone or ring,
 * has no contact with it.
 * ------------------------------------------------------------------------- */

enum { DEM_SURF_CYLINDER = 1, DEM_SURF_CONE = 2, DEM_SURF_DISK = 3, DEM_SURF_RING = 4 };

typedef struct dem_surface {
    int32_t kind;       /* DEM_SURF_*                                              */
    int32_t enabled;    /* 0: ignored (e.g. the plug of an opened orifice)          */
    double axis[2];     /* (x, y) of the vertical axis (m)                          */
    double z0, z1;      /* heights (m): cylinder and cone z0 < z1; disk, ring: z0   */
    double r0, r1;      /* radii (m) > 0: r0 (cone: at z0), r1 the cone's at z1     */
    double mu;          /* friction coefficient of a contact with the surface (the
                           paper lists particle-wall friction apart); < 0: that of
                           the particle's own material                              */
} dem_surface;

/* Set the surfaces of system `sys` (count <= its n_surf; host array).  The
 * tangential history of a surface whose record changed is cleared (enabling
 * or disabling one keeps the others').  Enqueued; DEM_ERR_ARG for a bad record
 * or count. */
int dem_set_surfaces(dem_ctx *ctx, int32_t sys, int32_t count, const dem_surface *surf);

/* Surface contact history, for checking and for resuming a run (synchronise;
 * host arrays).  Export: the tangential history that every live sphere
 * stored with a surface of its system (its surface contacts of the last
 * force evaluation), as (id, surface index k < count of its system, xi [3])
 * sorted by (id, k); *count receives the total even when it exceeds cap.
 * Import: replaces every sphere's surface history with the given records
 * (the others zero; a record of zeros is the same as none); an id that is
 * not live or an index beyond its system's surfaces is DEM_ERR_ARG. */
int dem_export_surface_history(dem_ctx *ctx, const dem_state *s, int32_t *id, int32_t *surf, double *xi, int64_t cap,
                               int64_t *count);
int dem_import_surface_history(dem_ctx *ctx, const dem_state *s, int64_t count, const int32_t *id,
                               const int32_t *surf, const double *xi);

/* ---------------------------------------------------------------------------
 * Insertion and deletion at the boundary of the fine region (Sec. 2.3).
 *
 * The paper measures the coarse particles' mass flow and velocity per cell of
 * the fine region's boundary surface, Favre-averages the velocity, inserts
 * fine particles cell by cell by simple sequential inhibition (SSI) and
 * removes fine particles that leave the region.  One dem_exchange call does
 * one such event on one system of the context (readings of the repository's
 * design notes):
 *   1. budget: with interval > 0 each boundary cell c gains the inflowing
 *      mass max(0, nrm . P_c) / slab * interval, P_c the momentum sum of the
 *      fields given (the coarse level's fields on the boundary cells, of
 *      dem_cell_fields);
 *   2. removal: every live sphere of the system whose centre has
 *      (x nrm_x + y nrm_y) + z nrm_z < face, or the same with out_nrm and
 *      out_face when out_nrm is not zero, is removed, with its history;
 *   3. SSI: candidate k (in the given order) is accepted iff its mass
 *      (4/3) pi rho r^3 is at most its cell's remaining budget and it
 *      overlaps neither a kept sphere nor a candidate accepted before it:
 *      d^2 < (r_k + r_j)^2 with d^2 = (dx dx + dy dy) + dz dz, dx the
 *      minimum image on periodic axes; an accepted candidate's mass is taken
 *      from its cell's budget;
 *   4. the accepted candidates are appended after the live spheres in
 *      candidate order with ids M + 1, M + 2, ... (M the largest id of the
 *      context's live spheres before the call), the Favre velocity P_c / M_c
 *      of their cell (zero where the cell holds no mass), no spin, zero force,
 *      torque, external force and history;
 *   5. the system's neighbour list is rebuilt (the kept pairs keep their
 *      history, by id) and its forces are evaluated at the new state without
 *      a history update, as dem_forces(ctx, s, 0) would; the other systems of
 *      the context are not touched (their state and forces stay bit for bit
 *      as they were).
 * ------------------------------------------------------------------------- */

typedef struct dem_exchange_params {
    double nrm[3];      /* unit normal of the boundary face, pointing into the fine region       */
    double face;        /* the region is x . nrm >= face; spheres below are removed               */
    double slab;        /* height of the inflow slab on the coarse side (m), > 0 when interval > 0 */
    double interval;    /* coupling interval (s); 0: no budget top-up (step 1 skipped)             */
    int64_t ncell;      /* boundary cells: rows of fields, entries of budget, range of cand_cell   */
    double out_nrm[3];  /* a second half-space x . out_nrm >= out_face bounding the region (an    */
    double out_face;    /*   outlet, e.g. below a silo's orifice); out_nrm = 0: none              */
} dem_exchange_params;

/* One insertion and deletion event on system `sys` (synchronises).
 *   fields     device [DEM_NFIELDS][ncell]: the coarse level's cell fields
 *              (DEM_F_MASS and DEM_F_MOM rows are read);
 *   budget     device [ncell], in/out: the mass each boundary cell may still
 *              insert (carried over between calls by the caller);
 *   ncand      candidates, 0 .. 2^20; cand_x device [3][ncand] positions (on
 *              periodic axes inside the box [lo, hi)), cand_r [ncand] radii in
 *              (0, r_max], cand_type [ncand] material indices, cand_cell
 *              [ncand] boundary cells in [0, ncell);
 *   accepted   device [ncand], out: 1 for an accepted candidate, else 0;
 *   counts     host int64[3], out: inserted, removed, live spheres after.
 * Requires the forces of the current state (the list then matches the
 * positions): DEM_ERR_STATE otherwise.  DEM_ERR_ARG for a bad candidate or
 * parameter, DEM_ERR_CAPACITY when the accepted spheres do not fit the
 * system's free slots or the candidates the workspace's scratch; on any
 * error nothing is changed (budget and accepted included). */
int dem_exchange(dem_ctx *ctx, const dem_state *s, int32_t sys, const dem_exchange_params *p, const double *fields,
                 double *budget, int64_t ncand, const double *cand_x, const double *cand_r, const int32_t *cand_type,
                 const int32_t *cand_cell, int32_t *accepted, int64_t counts[3]);

/* Live particles of system `sys` (host copy, no device work). */
int dem_live_count(dem_ctx *ctx, int32_t sys, int64_t *n);

/* ---------------------------------------------------------------------------
 * Material parameters and gradients with respect to them.
 *
 * The per-type E, e and mu enter the contact law through Eq. (6) (stiffnesses
 * from E* and G*, damping from beta(e)) and Eq. (5) (the Coulomb cap).  The
 * adjoint calls below give dL/dE, dL/de and dL/dmu of a scalar L of the
 * final state of a rollout (reverse mode, hand-written for the kernels).
 * ------------------------------------------------------------------------- */

/* Replace the materials of system `sys` (ntypes entries, as in its
 * configuration); the folded coefficients are recomputed and uploaded.  rho
 * must be unchanged (masses are fixed at dem_reset): DEM_ERR_ARG otherwise,
 * or for invalid values.  Synchronises. */
int dem_set_materials(dem_ctx *ctx, int32_t sys, const dem_material *mat, int32_t ntypes);

typedef struct dem_adjoint dem_adjoint;   /* opaque: rollout checkpoints and adjoint state */

/* Device bytes of the adjoint workspace of a rollout of nsteps steps with
 * checkpoints every `window` steps (1..4096) on a context of one system
 * (DEM_ERR_ARG for a batch).  max_windows bounds the number of windows: a
 * list rebuild ends a window early, so a rollout can need more than
 * ceil(nsteps / window); 0 selects 2 ceil(nsteps / window) + 1.
 * kslots (1..k_max, 0 = k_max): the tangential-history slots per particle
 * that the checkpoints and stored evaluation inputs hold, i.e. the longest
 * neighbour row the rollout may meet; the rollout and dem_forces_vjp return
 * DEM_ERR_CAPACITY when a list (the current one, or one built during the
 * rollout) has a longer row.  Rows hold the neighbours within the skin, so
 * a dense packing needs about 12, far fewer than a k_max sized for the
 * densest case.
 * keep = 0: checkpoints at window starts, each window recomputed by the
 * backward; memory (max_windows + window) x (128 + 32 kslots) bytes per
 * particle.  keep = 1: the inputs of every step are stored by the forward and
 * nothing is recomputed; memory (nsteps + 2) x (128 + 32 kslots) bytes per
 * particle.  Both: plus (max_windows + 1) x (28 + 4 kslots) bytes per
 * particle for the lists. */
int dem_adjoint_workspace_size(dem_ctx *ctx, int64_t nsteps, int32_t window, int32_t max_windows, int32_t keep,
                               int32_t kslots, size_t *bytes);

/* Bind an adjoint to a context and a caller-owned device workspace (256-byte
 * aligned, at least the size above for the same arguments, untouched until
 * dem_adjoint_destroy). */
int dem_adjoint_init(dem_ctx *ctx, int64_t nsteps, int32_t window, int32_t max_windows, int32_t keep,
                     int32_t kslots, void *workspace, size_t bytes, dem_adjoint **out);

/* The rollout: the force evaluation of the current state without history
 * update (as dem_forces(ctx, s, 0)), then nsteps steps bit-identical to
 * dem_step, run in windows of at most `window` steps with a checkpoint of the
 * packed state and the history at the start of each.  A list rebuild happens
 * only between windows (a rebuild request ends the window), so the contact
 * topology is fixed inside every window.  On return s holds the final state
 * (permuted by the rebuilds, as after dem_step).  DEM_ERR_CAPACITY when more
 * than max_windows windows are needed.  Synchronises once per window.  With
 * keep the steps are run by the evaluation kernel of the reverse pass, same
 * arithmetic and order, storing every step's inputs; the contact counters of
 * dem_stats are then not advanced. */
int dem_rollout_forward(dem_adjoint *adj, const dem_state *s);

/* Reverse mode of the last dem_rollout_forward (no other stepping in
 * between: DEM_ERR_STATE).  Inputs: gx, gv, gw = dL/dx, dL/dv, dL/dw of the
 * final state, device [3][n] in the final order.  Outputs: ax0, av0, aw0 =
 * dL/d(initial x, v, w), device [3][n] in the order of the first list build,
 * whose ids go to ids0 (device [n], may be NULL); grad = host [3][ntypes]:
 * dL/dE_t, then dL/de_t, then dL/dmu_t.  Each window is recomputed from its
 * checkpoint and reversed step by step; sums over particles are taken in a
 * fixed order, so results are reproducible (and equal with and without keep).
 * Synchronises. */
int dem_rollout_backward(dem_adjoint *adj, const dem_state *s, const double *gx, const double *gv, const double *gw,
                         double *ax0, double *av0, double *aw0, int32_t *ids0, double *grad);

/* Reverse mode of one force evaluation without history update (dem_forces(ctx,
 * s, 0)) at the current state and list: fb, tb = dL/df, dL/dt (device [3][n])
 * -> xb, vb, wb = dL/dx, dL/dv, dL/dw (device [3][n]) and grad (host
 * [3][ntypes], as above).  Uses the adjoint workspace.  Synchronises. */
int dem_forces_vjp(dem_adjoint *adj, const dem_state *s, const double *fb, const double *tb, double *xb, double *vb,
                   double *wb, double *grad);

/* Reverse mode of dem_integrate (the velocity-Verlet halves of Eq. (1)-(2)):
 * from the adjoints xb, vb, wb of the positions, velocities and spins that
 * dem_integrate(ctx, s, phase) writes, the adjoints of its inputs, per live
 * particle with dt of its system and m, I as fixed at dem_reset:
 *   phase 0 (v' = v + dt/2 f/m, w' = w + dt/2 t/I, x' = x + dt v' wrapped
 *   into the box): x_in = xb, v_in = vb + dt xb, w_in = wb,
 *   f_in = dt/2 (v_in / m), t_in = dt/2 (wb / I);
 *   phase 1 (v' = v + dt/2 f/m, w' = w + dt/2 t/I): x_in = xb, v_in = vb,
 *   w_in = wb, f_in = dt/2 (vb / m), t_in = dt/2 (wb / I).
 * The wrap shifts by a box length and passes the adjoint through; no material
 * parameter enters the integration, so there is no parameter gradient.  All
 * arrays device [3][n] in the context's current order; free slots get zeros;
 * outputs must not overlap inputs.  DEM_ERR_STATE before dem_reset,
 * DEM_ERR_ARG for another phase or a NULL array.  Enqueued. */
int dem_integrate_vjp(dem_ctx *ctx, const dem_state *s, int32_t phase, const double *xb, const double *vb,
                      const double *wb, double *x_in, double *v_in, double *w_in, double *f_in, double *t_in);

/* Threads per particle in the evaluation and reverse kernels: 4 (default) or
 * 8.  Sums over a particle's row are taken per lane and then over the lanes
 * in order, so results are reproducible for a given choice. */
int dem_adjoint_set_lanes(dem_adjoint *adj, int32_t lanes);

/* out[0] windows of the last forward, out[1] list rebuilds in it, out[2]
 * workspace bytes, out[3] max_windows. */
int dem_adjoint_info(dem_adjoint *adj, int64_t out[4]);

/* Release the adjoint (host memory only). */
int dem_adjoint_destroy(dem_adjoint *adj);

const char *dem_last_error(const dem_ctx *ctx);

/* Release the context (host memory only; the workspace stays the caller's). */
int dem_destroy(dem_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* DEM_H */
