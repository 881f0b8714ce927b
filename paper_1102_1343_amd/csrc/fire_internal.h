// Internal declarations shared by the kernels and the C ABI layer of the
// fire-mesh step library (gfx950).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "fire.h"

namespace fire {

// Fused step kernel geometry.  A work-group owns a tile of tile_x x tile_y
// fire cells and stages a frame of (tile_x + 6) x (tile_y + 6) cells in LDS:
// three halo rings, because the two Heun stages each reach one cell and the
// fuel-fraction stencil one more.  Frame rows are 128 lanes wide (two
// wave64s); kNR frame rows are processed at once.
constexpr int kFW = 128;
constexpr int kNR = 4;
constexpr int kHalo = 3;
constexpr int kFHMax = 48;
constexpr int kTileXMax = kFW - 2 * kHalo;      // 122
constexpr int kTileYMax = kFHMax - 2 * kHalo;   // 42
constexpr int kTileYMax64 = 26;                  // FP64 frames must fit LDS
constexpr int kBlock = kFW * kNR;

// coefficient table columns (one row per fuel category)
enum { kS0, kR0, kB, kC, kD, kE, kM, kTf, kCh, kCq, kNCoef };

// status word bits (same values as FIRE_STATUS_*)
constexpr int kStBoundary = FIRE_STATUS_BOUNDARY;
constexpr int kStNonfinite = FIRE_STATUS_NONFINITE;

// Per-launch arguments.  For one domain the domain fields describe it; for an
// ensemble they are overwritten per tile from the domain table.
struct StepArgs {
    int32_t nx, ny;
    int32_t tile_x, tile_y;
    int32_t tiles_x, ntiles, per_xcd;   // ntiles: total tiles of the launch
    int32_t sr_x, sr_y, nax, nay;
    int32_t ncat, guard, visc_mode, nign, mark_step;   // mark_step: see StepBuffers::mark
    int32_t tile_cap, ign_rows;   // plain step: see IgnSetLayout
    double dx, dy;
    double rdx, rdy;     // 1/dx, 1/dy
    double t, dt;        // t unused by the ensemble kernel (device time)
    double eps, ros_cap;
};

// One ignition's geometry at a time t (Sect. 4.4): the segment start in
// double, so node offsets are formed exactly from global coordinates and
// psi_g at a node is the same in every tile that touches the node; the
// segment vector, its share of the projection (e / |e|^2), the current
// radius, start time, drip-torch time per unit length, 1 / S_g and t.
template <typename T> struct IgnGeo {
    double ax, ay;
    T ex, ey, exL, eyL, rad, tg, lenv, invS, t, pad;
};

// Geometry of a domain's ignitions for one step, formed once per step by a
// small kernel ahead of the step kernel (on = active at that time).
template <typename T> struct IgnTable {
    IgnGeo<T> g[FIRE_MAX_IGNITIONS];
    int32_t on[FIRE_MAX_IGNITIONS];
};
// bytes reserved per domain for its table (room for either precision)
constexpr size_t kIgnTableBytes = (sizeof(IgnTable<double>) + 255) / 256 * 256;

// Per-tile ignition set-up of a single domain's step, formed with the
// geometry ahead of the step kernel, so the step reads it with scalar loads:
//  * use[tile] (tile < tile_cap), 2 bits per ignition g at bit 2g: 0 the
//    ignition cannot change the tile's frame, 1 it can lower psi but lights
//    no node there (psi_g > 0 on the whole frame), 2 it may light nodes;
//    use[tile_cap] is the word for tiles past the capacity (2 for every
//    active ignition);
//  * lb[tile][g], a lower bound of psi_g over the tile's frame;
//  * rows[g][gy + kHalo] and rows[FIRE_MAX_IGNITIONS + g][gy + kHalo], the
//    node-row offsets py and by of global row gy, for gy in
//    [-kHalo, ny + kFHMax - kHalo) (every frame row of every tile).
// tile_cap is the tile count at the mesh's default tile shape.
struct IgnSetLayout {
    size_t use, lb, rows, total;
};
inline IgnSetLayout ign_set_layout(int tile_cap, int ny, size_t esz) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    IgnSetLayout L;
    L.use = 0;
    L.lb = up((size_t)(tile_cap + 1) * sizeof(uint32_t));
    L.rows = L.lb + up((size_t)tile_cap * FIRE_MAX_IGNITIONS * esz);
    L.total = L.rows + up((size_t)2 * FIRE_MAX_IGNITIONS * (ny + kFHMax) * esz);
    return L;
}

// One member of an ensemble (device table row).
struct EnsDomain {
    int32_t nx, ny, tiles_x, tile0;     // tile0: first work-list tile of the domain
    int32_t nax, nay, nign, pad;
    double dx, dy, rdx, rdy;
    int64_t cell_off, atm_off;          // element offsets into the concatenated arrays
    double t_ign_lo, t_ign_hi;          // ignition_window() of the member's ignitions
};

// Device-side clock of an ensemble: model time and which psi buffer holds
// the current state, so that a step enqueues the same launches every time
// (graph capture).
struct EnsClock {
    double t;
    int32_t cur;
    int32_t pad;
};

struct StepBuffers {
    const void *psi_in;
    void *psi_out;
    void *tign;
    void *frac;
    const void *u, *v, *dzdx, *dzdy;
    const uint8_t *cat;
    const void *coef;
    void *fsens, *flat;
    int *status;
    const fire_ignition *ign;           // device ignition records: one domain's, or
                                        // FIRE_MAX_IGNITIONS per ensemble member
    void *ign_tab;                      // kIgnTableBytes per domain: the step's
                                        // ignition geometry (IgnTable)
    int32_t ndom;                       // domains of an ensemble launch
    size_t ncells;                      // cells in the (concatenated) arrays
    const EnsDomain *ens_doms;          // non-null for an ensemble launch; then
    const int32_t *ens_tile_dom;        // psi_in / psi_out are the two buffers and
    const EnsClock *ens_clock;          // the clock says which is current
    int32_t *ens_counters;              // 8 work counters (resident work-groups)
    int32_t ens_slots;                  // > 0: resident work-groups (k_ens_persist)
    void *rec_p0, *rec_b;               // non-null: a replay that writes psi^{n+1}, psi'
                                        // and psi* only (one domain)
    int32_t *mark;                      // non-null (plain step): mark[i] = mark_step at
                                        // each node whose ignition time the step sets
    void *ign_set;                      // plain step: the per-tile ignition set-up
                                        // (IgnSetLayout), null for an ensemble
};

}  // namespace fire

// A single-domain context (host side).  The arena holds, at these offsets,
// the coefficient table, the fuel staging copy, the ignition records, the
// status word, psi (two buffers), t_i and F.
struct fire_ctx {
    fire_mesh mesh;
    fire_params prm;
    int ncat;
    int nign;
    fire_ignition ign[FIRE_MAX_IGNITIONS];
    const uint8_t *cat;
    const void *dzdx, *dzdy;
    char *arena;
    size_t off_coef, off_fuel, off_ign, off_geo, off_iset, off_status, off_psi[2], off_tign,
        off_frac;
    int tile_cap;          // tiles at the default tile shape (IgnSetLayout)
    int cur;               // index of the current psi buffer
    double t;              // model time of the current state
    hipStream_t stream;
    int tile_x, tile_y;
    int stopped;           // FIRE_ERR_BOUNDARY / FIRE_ERR_NONFINITE once the stop
                           // policy has seen that status bit, else 0
    // Stop policy: after each step the status word is copied to pinned host
    // memory (slot nstep % 2) and an event is recorded; the next call reads
    // the copies that are complete, waiting only for the one two steps back.
    int32_t *host_status;  // hipHostMalloc'd, 2 slots (null under policy 1)
    hipEvent_t ev[2];
    int ev_valid[2];
    long nstep;
    // Set by a differentiable run's recording forward for the duration of a
    // step: the step index stored where that step sets an ignition time.
    int32_t *mark;
    int32_t mark_step;
};

namespace fire {

// launchers (return hipError_t of the launch)
hipError_t launch_step(int dtype, const StepArgs &a, const StepBuffers &b, hipStream_t s);
hipError_t launch_coef(int dtype, const fire_fuel *fuels_dev, int ncat, double wind_cap,
                       void *coef_dev, hipStream_t s);
hipError_t launch_fill(int dtype, void *psi, void *tign, void *frac, size_t n, double psi0,
                       hipStream_t s);
hipError_t launch_ros_eval(int dtype, const void *coef, int ncat, double ros_cap,
                           const uint8_t *cat, const void *un, const void *tn, void *S,
                           int64_t n, hipStream_t s);
hipError_t launch_coef_to_f64(int dtype, const void *coef, double *out, int n, hipStream_t s);
hipError_t launch_advance_clock(EnsClock *c, double dt, hipStream_t s);
// resident work-groups of the ensemble step for this tile height (0: query failed)
int persist_slots(int dtype, int tile_y, int ncat, size_t ncells);

// ---- host helpers shared by the single-domain and ensemble ABI layers
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline size_t esize(const fire_mesh *m) { return m->dtype == FIRE_F64 ? 8 : 4; }
bool mesh_ok(const fire_mesh *m);
bool params_ok(const fire_params *p);
bool fuels_ok(const fire_fuel *cats, int ncat);
bool ignitions_ok(const fire_ignition *ign, int nign);
void default_tile(const fire_mesh *m, int *tx, int *ty);
bool tile_ok(const fire_mesh *m, int tile_x, int tile_y);
// [lo, hi] outside which none of the ignitions is active (the activity test
// of the step kernel, in the same double arithmetic); lo > hi when n = 0.
void ignition_window(const fire_ignition *ign, int n, double *lo, double *hi);
hipError_t step_raw(fire_ctx *c, const void *psi_in, void *psi_out, void *tign, void *frac,
                    const void *u, const void *v, double t, double dt, void *flux_sens,
                    void *flux_lat, int *status, void *rec_p0 = nullptr, void *rec_b = nullptr,
                    hipStream_t stream = nullptr);   // null: the context's stream

}  // namespace fire
