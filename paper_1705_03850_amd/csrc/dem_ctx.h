// dem_ctx.h -- host-side context of libdem.so (internal): workspace layout,
// the context struct and the helpers shared by the host translation units.
#pragma once

#include <cstring>
#include <string>
#include <vector>

#include "../../include/dem.h"
#include "dem_kernels.h"

namespace dem {
namespace host {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t sys, coef, rho, flags, m, inv_m, inv_I, disp, xiw, frame, dead, fext;
    size_t nbr[2], cnt[2], xi[2], mask[2], ids[2];
    size_t cell_of, rank, order, cell_count, cell_start, scan_partial, shadow_d, shadow_i;
    size_t pos[2], vel[2], spin[2], im, sel, lcur, tile0, mtile0, msys, mlevel;
    size_t surf, sxi, smask, shadow_s;   // surfaces (sxi, smask, shadow_s: 0 without any)
    size_t total;
};

struct Geometry {
    std::vector<SysDesc> sys;
    std::vector<PairCoef> coef;
    std::vector<double> rho;
    std::vector<dem_material> mat;   // per type, all systems (host copy of the parameters)
    std::vector<int32_t> surf_cap;   // surfaces reserved per system
    std::vector<Surf> surf;          // [nsys * kMaxSurf] host copy of the surface table
    int32_t nsurf_slots = 0;         // surface history slots per particle (the largest reservation)
    int64_t n = 0, ncell = 0;
    int32_t kmax = 0, block = 128;
};

constexpr int kKinds = 4;  // timed kernel classes: phase 0, forces, phase 1, list rebuild

struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    const void *key[10] = {nullptr};
    int chunk = 0;
    int count = 0;
};

}  // namespace host
}  // namespace dem

struct dem_ctx {
    dem::host::Geometry geo;
    dem::host::Layout lay;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    dem::SysDesc *d_sys = nullptr;
    dem::PairCoef *d_coef = nullptr;
    double *d_rho = nullptr;
    dem::Flags *d_flags = nullptr;
    dem::Flags *h_flags = nullptr;   // pinned host copy for read_flags (null: a pageable copy)
    dem::List lists[2];
    // host-side state machine
    bool masses = false, have_list = false, list_current = false, binned = false, frame_identity = true;
    bool forces_valid = false;
    bool fext_on = false;            // external forces are added to the force evaluations
    bool multirate = false;          // systems step every SysDesc::stride substeps
    bool win_on = false;             // rebuild kernels limited to win: particles [0], [1), cells [2], [3)
    int64_t win[4] = {0, 0, 0, 0};
    int32_t max_stride = 1;
    int64_t step_counter = 0;
    // options
    bool use_graph = false, count = true;
    int chunk = 64;
    int64_t grid_cap = 0;   // 0: resident capacity, set at init
    int lanes = 4;
    int cus = 256;
    int64_t ntiles_b = 0;            // tiles of the batch step (each within one system)
    dem::host::GraphSlot graphs[8];          // replay graphs of 2^(k+3) fused steps
    hipGraphExec_t cpl_exec = nullptr;       // one coupled interval (dem_step_coupled)
    std::vector<char> cpl_key;               // what it was captured for
    double gap_avg = 1e9;         // running estimate of steps between rebuilds
    int64_t since_rebuild = 0;
    // per-kernel timing with HIP events (non-graph stepping only)
    bool timing = false;
    std::vector<hipEvent_t> ev;      // pairs (start, stop) recorded in this chunk
    std::vector<int> ev_kind;        // kernel class of each pair
    std::vector<int> ev_count;       // launches between the two events of each pair
    int ev_used = 0;
    double t_ms[dem::host::kKinds] = {0, 0, 0, 0};
    int64_t t_n[dem::host::kKinds] = {0, 0, 0, 0};
    std::string err;
    int static_dev = -1;             // >= 0: the workspace is that device's static array (dem_init_noalloc)
};

namespace dem {
namespace host {

#define HIPCALL(c, expr)                                            \
    do {                                                            \
        hipError_t _e = (expr);                                     \
        if (_e != hipSuccess) return hip_fail((c), _e, #expr);      \
    } while (0)

int fail(dem_ctx *c, int code, const std::string &msg);
int hip_fail(dem_ctx *c, hipError_t e, const char *what);
KArgs kargs(dem_ctx *c, const dem_state *s);
int check_state(dem_ctx *c, const dem_state *s);
int read_flags(dem_ctx *c, Flags &h);
int flag_error(dem_ctx *c, const Flags &h);
int upload_tiles(dem_ctx *c);
int do_bin(dem_ctx *c, const dem_state *s, bool all);
int do_neighbors(dem_ctx *c, const dem_state *s, bool clear_sel = true);
// The current list buffer of system sy (reads the device's choice; synchronises).
int live_list(dem_ctx *c, int sy, List &out);
// Stepping pieces shared by dem_step and dem_step_coupled (dem_api.hip).
int rebuild_at(dem_ctx *c, const dem_state *s, int64_t qa);
int step_loop(dem_ctx *c, const dem_state *s, int64_t nsteps, int64_t base, int64_t q, Flags &h);
int collect_times(dem_ctx *c);
void note_rebuild(dem_ctx *c, int64_t ran);
void note_steps(dem_ctx *c, int64_t ran);
// E > 0, -1 < nu < 0.5, rho > 0, 0 < e <= 1, mu >= 0, all finite.
bool material_ok(const dem_material &m);
// Folded Eq. (6) coefficients of a pair of materials.
PairCoef pair_coef(const dem_material &a, const dem_material &b);

}  // namespace host
}  // namespace dem
