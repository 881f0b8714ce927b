// C ABI of the fire-mesh step library: argument checking, the state arena
// layout, the fire time bookkeeping and kernel launches.  Every piece of the
// method's arithmetic runs in the kernels of fire_kernels.hip.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "fire_internal.h"

using namespace fire;

namespace fire {

bool mesh_ok(const fire_mesh *m) {
    if (!m) return false;
    if (m->nx < 2 || m->ny < 2) return false;
    if ((int64_t)m->nx * m->ny > ((int64_t)1 << 31)) return false;
    if (!(m->dx > 0.0) || !(m->dy > 0.0) || !std::isfinite(m->dx) || !std::isfinite(m->dy))
        return false;
    if (m->sr_x < 1 || m->sr_x > kTileXMax || m->sr_y < 1 || m->sr_y > kTileYMax64) return false;
    return m->dtype == FIRE_F32 || m->dtype == FIRE_F64;
}

bool params_ok(const fire_params *prm) {
    if (!prm) return false;
    if (!(prm->viscosity >= 0.0) || !std::isfinite(prm->viscosity)) return false;
    if (!(prm->wind_cap > 0.0) || !(prm->ros_cap > 0.0) || !std::isfinite(prm->t0)) return false;
    if (prm->guard_width < 0 || (prm->boundary_policy != 0 && prm->boundary_policy != 1) ||
        (prm->viscosity_mode != 0 && prm->viscosity_mode != 1))
        return false;
    return true;
}

bool fuels_ok(const fire_fuel *cats, int ncat) {
    if (!cats || ncat < 1 || ncat > 256) return false;
    for (int k = 0; k < ncat; k++) {
        const fire_fuel &f = cats[k];
        if (!(f.ros_mult >= 0.0)) return false;
        if (!(f.tf > 0.0) && !(f.weight > 0.0)) return false;
        if (!f.ichap && !(f.fgi > 0.0 && f.fueldepthm > 0.0 && f.savr > 0.0 && f.fuelmce > 0.0 &&
                          f.fueldens > 0.0 && f.se > 0.0 && f.fuelmc_g >= 0.0))
            return false;
    }
    return true;
}

bool ignitions_ok(const fire_ignition *ign, int nign) {
    if (nign < 0 || nign > FIRE_MAX_IGNITIONS || (nign > 0 && !ign)) return false;
    for (int g = 0; g < nign; g++) {
        const fire_ignition &r = ign[g];
        if (!(r.ros > 0.0) || !(r.radius >= 0.0) || !std::isfinite(r.radius) ||
            !std::isfinite(r.t_start))
            return false;
        if ((r.vx != 0.0 || r.vy != 0.0) && !(r.t_end >= r.t_start)) return false;
    }
    return true;
}

// default tile: widest multiple of sr_x that fits the frame, and the
// tallest multiple of sr_y up to 20 rows; when sr_y > 20 the one multiple
// sr_y itself (mesh_ok keeps sr_y within the FP64 frame limit)
void default_tile(const fire_mesh *m, int *tx, int *ty) {
    *tx = (kTileXMax / m->sr_x) * m->sr_x;
    const int ymax = m->dtype == FIRE_F64 ? kTileYMax64 : kTileYMax;
    int best = 0;
    for (int h = m->sr_y; h <= ymax; h += m->sr_y)
        if (h <= 20 || best == 0) best = h;
    *ty = best;
}

void ignition_window(const fire_ignition *ign, int n, double *lo, double *hi) {
    *lo = 1.0;
    *hi = 0.0;
    for (int g = 0; g < n; g++) {
        const fire_ignition &q = ign[g];
        const bool torch = (q.vx != 0.0 || q.vy != 0.0);
        const double tend = torch ? q.t_end : q.t_start;
        const double grow = std::isinf(q.ros) ? 0.0 : q.radius / q.ros;
        const double last = tend + grow;
        if (g == 0 || q.t_start < *lo) *lo = q.t_start;
        if (g == 0 || last > *hi) *hi = last;
    }
}

bool tile_ok(const fire_mesh *m, int tile_x, int tile_y) {
    const int ymax = m->dtype == FIRE_F64 ? kTileYMax64 : kTileYMax;
    if (tile_x < 1 || tile_x > kTileXMax || tile_x % m->sr_x != 0) return false;
    if (tile_y < 1 || tile_y > ymax || tile_y % m->sr_y != 0) return false;
    return true;
}

}  // namespace fire

namespace {

struct Layout {
    size_t coef, fuel, ign, geo, iset, status, psi0, psi1, tign, frac, total;
    int tile_cap;
};

// tiles at the mesh's default tile shape: the capacity of the per-tile
// ignition set-up
int default_tiles(const fire_mesh *m) {
    int tx, ty;
    default_tile(m, &tx, &ty);
    return ((m->nx + tx - 1) / tx) * ((m->ny + ty - 1) / ty);
}

Layout layout(const fire_mesh *m, int ncat) {
    const size_t n = (size_t)m->nx * m->ny, e = esize(m);
    Layout L;
    size_t o = 0;
    L.coef = o;
    o = align_up(o + (size_t)ncat * kNCoef * e);
    L.fuel = o;
    o = align_up(o + (size_t)ncat * sizeof(fire_fuel));
    L.ign = o;
    o = align_up(o + FIRE_MAX_IGNITIONS * sizeof(fire_ignition));
    L.geo = o;
    o = align_up(o + kIgnTableBytes);
    L.tile_cap = default_tiles(m);
    L.iset = o;
    o = align_up(o + ign_set_layout(L.tile_cap, m->ny, e).total);
    L.status = o;
    o = align_up(o + 64);
    L.psi0 = o;
    o = align_up(o + n * e);
    L.psi1 = o;
    o = align_up(o + n * e);
    L.tign = o;
    o = align_up(o + n * e);
    L.frac = o;
    o = align_up(o + n * e);
    L.total = o;
    return L;
}

int hip_fail(hipError_t e) { return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP; }

void *state_ptr(fire_ctx *c, size_t off) { return c->arena + off; }

}  // namespace

namespace fire {
// One step of the context's mesh on explicit buffers (the context's own
// arena for fire_step, replay buffers for the adjoint).
hipError_t step_raw(fire_ctx *c, const void *psi_in, void *psi_out, void *tign, void *frac,
                    const void *u, const void *v, double t, double dt, void *flux_sens,
                    void *flux_lat, int *status, void *rec_p0, void *rec_b,
                    hipStream_t stream) {
    const fire_mesh &m = c->mesh;
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = m.nx;
    a.ny = m.ny;
    a.tile_x = c->tile_x;
    a.tile_y = c->tile_y;
    a.tiles_x = (m.nx + c->tile_x - 1) / c->tile_x;
    const int tiles_y = (m.ny + c->tile_y - 1) / c->tile_y;
    a.ntiles = a.tiles_x * tiles_y;
    a.per_xcd = (a.ntiles + 7) / 8;
    a.sr_x = m.sr_x;
    a.sr_y = m.sr_y;
    a.nax = (m.nx + m.sr_x - 1) / m.sr_x;
    a.nay = (m.ny + m.sr_y - 1) / m.sr_y;
    a.ncat = c->ncat;
    a.guard = c->prm.guard_width;
    a.visc_mode = c->prm.viscosity_mode;
    double lo, hi;   // no ignition is active outside [lo, hi]: skip the loop
    ignition_window(c->ign, c->nign, &lo, &hi);
    a.nign = (t >= lo && t <= hi) ? c->nign : 0;
    a.dx = m.dx;
    a.dy = m.dy;
    a.rdx = 1.0 / m.dx;
    a.rdy = 1.0 / m.dy;
    a.t = t;
    a.dt = dt;
    a.eps = c->prm.viscosity;
    a.ros_cap = c->prm.ros_cap;

    StepBuffers b;
    std::memset(&b, 0, sizeof(b));
    b.psi_in = psi_in;
    b.psi_out = psi_out;
    b.tign = tign;
    b.frac = frac;
    b.u = u;
    b.v = v;
    b.dzdx = c->dzdx;
    b.dzdy = c->dzdy;
    b.cat = c->cat;
    b.coef = state_ptr(c, c->off_coef);
    b.fsens = flux_sens;
    b.flat = flux_lat;
    b.status = status;
    b.ign = (const fire_ignition *)state_ptr(c, c->off_ign);
    b.ign_tab = state_ptr(c, c->off_geo);
    b.ndom = 1;
    b.ncells = (size_t)m.nx * m.ny;
    b.ens_doms = nullptr;
    b.ens_tile_dom = nullptr;
    b.ens_clock = nullptr;
    b.rec_p0 = rec_p0;
    b.rec_b = rec_b;
    b.mark = rec_p0 ? nullptr : c->mark;
    a.mark_step = c->mark_step;
    a.tile_cap = c->tile_cap;
    a.ign_rows = m.ny + kFHMax;
    b.ign_set = state_ptr(c, c->off_iset);

    return launch_step(m.dtype, a, b, stream ? stream : c->stream);
}

}  // namespace fire

extern "C" {

int fire_abi_version(void) { return FIRE_ABI_VERSION; }

const char *fire_strerror(int code) {
    switch (code) {
    case FIRE_OK: return "ok";
    case FIRE_ERR_ARG: return "invalid argument";
    case FIRE_ERR_HIP: return "HIP runtime or kernel launch error";
    case FIRE_ERR_OOM: return "host allocation failed";
    case FIRE_ERR_BOUNDARY: return "fire reached the domain boundary guard ring";
    case FIRE_ERR_NONFINITE: return "non-finite level set or fuel fraction";
    case FIRE_ERR_STATE: return "call not allowed in the current context state";
    case FIRE_ERR_TOO_LARGE: return "input larger than the library's fixed-size buffer allows";
    default: return "unknown error";
    }
}

size_t fire_state_bytes(const fire_mesh *mesh, int32_t ncat) {
    if (!mesh_ok(mesh) || ncat < 1 || ncat > 256) return 0;
    return layout(mesh, ncat).total;
}

int fire_init(fire_ctx **out, const fire_mesh *mesh, const fire_fuel *cats, int32_t ncat,
              const uint8_t *fuel_cat, const void *dzdx, const void *dzdy,
              const fire_ignition *ign, int32_t nign, const fire_params *prm, void *state,
              size_t state_bytes, void *stream) {
    if (!out) return FIRE_ERR_ARG;
    *out = nullptr;
    if (!mesh_ok(mesh) || !fuels_ok(cats, ncat) || !fuel_cat || !dzdx || !dzdy ||
        !params_ok(prm) || !state || !ignitions_ok(ign, nign))
        return FIRE_ERR_ARG;
    if (((uintptr_t)state % kAlign) != 0) return FIRE_ERR_ARG;
    const Layout L = layout(mesh, ncat);
    if (state_bytes < L.total) return FIRE_ERR_ARG;

    fire_ctx *c = new (std::nothrow) fire_ctx();
    if (!c) return FIRE_ERR_OOM;
    c->mesh = *mesh;
    c->prm = *prm;
    c->ncat = ncat;
    c->nign = nign;
    for (int g = 0; g < nign; g++) c->ign[g] = ign[g];
    c->cat = fuel_cat;
    c->dzdx = dzdx;
    c->dzdy = dzdy;
    c->arena = (char *)state;
    c->off_coef = L.coef;
    c->off_fuel = L.fuel;
    c->off_ign = L.ign;
    c->off_geo = L.geo;
    c->off_iset = L.iset;
    c->tile_cap = L.tile_cap;
    c->off_status = L.status;
    c->off_psi[0] = L.psi0;
    c->off_psi[1] = L.psi1;
    c->off_tign = L.tign;
    c->off_frac = L.frac;
    c->cur = 0;
    c->t = prm->t0;
    c->stream = (hipStream_t)stream;
    c->stopped = 0;
    c->host_status = nullptr;
    c->ev[0] = c->ev[1] = nullptr;
    c->ev_valid[0] = c->ev_valid[1] = 0;
    c->mark = nullptr;
    c->mark_step = 0;
    c->nstep = 0;
    default_tile(mesh, &c->tile_x, &c->tile_y);
    if (!tile_ok(mesh, c->tile_x, c->tile_y)) {
        delete c;
        return FIRE_ERR_ARG;
    }
    if (prm->boundary_policy == 0) {
        // pinned host slots for the lagging status copies (host memory; the
        // library still allocates no device memory)
        void *hs = nullptr;
        if (hipHostMalloc(&hs, 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
            delete c;
            return FIRE_ERR_HIP;
        }
        c->host_status = (int32_t *)hs;
        c->host_status[0] = c->host_status[1] = 0;
        if (hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) != hipSuccess) {
            fire_destroy(c);
            return FIRE_ERR_HIP;
        }
    }

    // the fuel table goes through the arena (it may exceed kernel-argument
    // space); the copy is synchronous because cats is pageable host memory
    hipError_t e = hipMemcpyAsync(state_ptr(c, L.fuel), cats, sizeof(fire_fuel) * ncat,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && nign > 0)
        e = hipMemcpyAsync(state_ptr(c, L.ign), ign, sizeof(fire_ignition) * nign,
                           hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = launch_coef(mesh->dtype, (const fire_fuel *)state_ptr(c, L.fuel), ncat, prm->wind_cap,
                        state_ptr(c, L.coef), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(state_ptr(c, L.status), 0, 64, c->stream);
    double psi0 = prm->psi_init;
    if (!(psi0 > 0.0))
        psi0 = std::sqrt((mesh->nx * mesh->dx) * (mesh->nx * mesh->dx) +
                         (mesh->ny * mesh->dy) * (mesh->ny * mesh->dy));
    if (e == hipSuccess)
        e = launch_fill(mesh->dtype, state_ptr(c, L.psi0), state_ptr(c, L.tign),
                        state_ptr(c, L.frac), (size_t)mesh->nx * mesh->ny, psi0, c->stream);
    if (e != hipSuccess) {
        fire_destroy(c);
        return FIRE_ERR_HIP;
    }
    *out = c;
    return FIRE_OK;
}

namespace {

// Stop policy: the status a completed copy reports, as an error code (0 if
// neither bit is set).
int status_code(int32_t st) {
    if (st & FIRE_STATUS_BOUNDARY) return FIRE_ERR_BOUNDARY;
    if (st & FIRE_STATUS_NONFINITE) return FIRE_ERR_NONFINITE;
    return FIRE_OK;
}

// Reads the lagging status copies: the one of the step before the last is
// waited for (so at most one step is in flight beyond what has been checked),
// the last one only if it has completed.  Returns an error code to stop with,
// FIRE_OK, or FIRE_ERR_HIP.
int check_lagged(fire_ctx *c) {
    for (int back = 1; back >= 0; back--) {
        const long k = c->nstep - 1 - back;   // step whose copy sits in slot k % 2
        if (k < 0) continue;
        const int slot = (int)(k % 2);
        if (!c->ev_valid[slot]) continue;
        hipError_t e = back == 1 ? hipEventSynchronize(c->ev[slot]) : hipEventQuery(c->ev[slot]);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return FIRE_ERR_HIP;
        c->ev_valid[slot] = 0;
        const int code = status_code(c->host_status[slot]);
        if (code != FIRE_OK) return code;
    }
    return FIRE_OK;
}

}  // namespace

int fire_step(fire_ctx *c, const void *u, const void *v, double dt, void *flux_sens,
              void *flux_lat, fire_view *out) {
    if (!c || !u || !v || !flux_sens || !flux_lat) return FIRE_ERR_ARG;
    if (!(dt > 0.0) || !std::isfinite(dt)) return FIRE_ERR_ARG;
    if (c->stopped) return c->stopped;
    if (c->prm.boundary_policy == 0) {
        // Sect. 4.1: the run terminates when fire reaches the boundary.  The
        // condition is read from copies of the status word lagging by at most
        // one step, so the host never waits for the step it just enqueued.
        const int code = check_lagged(c);
        if (code == FIRE_ERR_HIP) return code;
        if (code != FIRE_OK) {
            c->stopped = code;
            return code;
        }
    }

    hipError_t e = step_raw(c, state_ptr(c, c->off_psi[c->cur]),
                            state_ptr(c, c->off_psi[1 - c->cur]), state_ptr(c, c->off_tign),
                            state_ptr(c, c->off_frac), u, v, c->t, dt, flux_sens, flux_lat,
                            (int *)state_ptr(c, c->off_status));
    if (e != hipSuccess) return FIRE_ERR_HIP;
    c->cur = 1 - c->cur;
    c->t += dt;
    if (out) {
        out->psi = state_ptr(c, c->off_psi[c->cur]);
        out->tign = state_ptr(c, c->off_tign);
        out->frac = state_ptr(c, c->off_frac);
        out->t = c->t;
    }
    if (c->prm.boundary_policy == 0) {
        const int slot = (int)(c->nstep % 2);
        e = hipMemcpyAsync(&c->host_status[slot], state_ptr(c, c->off_status), sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipEventRecord(c->ev[slot], c->stream);
        if (e != hipSuccess) return FIRE_ERR_HIP;
        c->ev_valid[slot] = 1;
    }
    c->nstep++;
    return FIRE_OK;
}

int fire_get_state(fire_ctx *c, fire_view *out) {
    if (!c || !out) return FIRE_ERR_ARG;
    out->psi = state_ptr(c, c->off_psi[c->cur]);
    out->tign = state_ptr(c, c->off_tign);
    out->frac = state_ptr(c, c->off_frac);
    out->t = c->t;
    return FIRE_OK;
}

int fire_set_state(fire_ctx *c, const void *psi, const void *tign, const void *frac, double t) {
    if (!c || !psi || !tign || !frac || !std::isfinite(t)) return FIRE_ERR_ARG;
    const size_t bytes = (size_t)c->mesh.nx * c->mesh.ny * esize(&c->mesh);
    hipError_t e = hipMemcpyAsync(state_ptr(c, c->off_psi[c->cur]), psi, bytes,
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(state_ptr(c, c->off_tign), tign, bytes, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(state_ptr(c, c->off_frac), frac, bytes, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(state_ptr(c, c->off_status), 0, 64, c->stream);
    if (e != hipSuccess) return FIRE_ERR_HIP;
    c->t = t;
    c->stopped = 0;
    c->ev_valid[0] = c->ev_valid[1] = 0;   // copies of the old status are not read
    return FIRE_OK;
}

int fire_status(fire_ctx *c) {
    if (!c) return FIRE_ERR_ARG;
    int32_t st = 0;
    hipError_t e = hipMemcpyAsync(&st, state_ptr(c, c->off_status), sizeof(st),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return FIRE_ERR_HIP;
    st &= FIRE_STATUS_BOUNDARY | FIRE_STATUS_NONFINITE;
    if (c->prm.boundary_policy == 0 && !c->stopped && status_code(st) != FIRE_OK)
        c->stopped = status_code(st);   // the stop policy holds from here on
    return st;
}

int fire_default_tile(const fire_mesh *mesh, int32_t *tile_x, int32_t *tile_y) {
    if (!mesh_ok(mesh) || !tile_x || !tile_y) return FIRE_ERR_ARG;
    int tx, ty;
    default_tile(mesh, &tx, &ty);
    if (!tile_ok(mesh, tx, ty)) return FIRE_ERR_ARG;
    *tile_x = tx;
    *tile_y = ty;
    return FIRE_OK;
}

int fire_coef(fire_ctx *c, double *out, int32_t ncat) {
    if (!c || !out || ncat != c->ncat) return FIRE_ERR_ARG;
    // widened into the fuel staging area (no longer needed after init; a
    // fuel record is larger than a row of doubles), then copied out
    static_assert(sizeof(fire_fuel) >= kNCoef * sizeof(double), "staging area too small");
    const int n = c->ncat * kNCoef;
    double *stage = (double *)state_ptr(c, c->off_fuel);
    hipError_t e = launch_coef_to_f64(c->mesh.dtype, state_ptr(c, c->off_coef), stage, n,
                                      c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, stage, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_fail(e);
}

int fire_ros_eval(fire_ctx *c, const uint8_t *cat, const void *un, const void *tn, void *S,
                  int64_t n) {
    if (!c || n < 0 || (n > 0 && (!cat || !un || !tn || !S))) return FIRE_ERR_ARG;
    if (n == 0) return FIRE_OK;
    return hip_fail(launch_ros_eval(c->mesh.dtype, state_ptr(c, c->off_coef), c->ncat,
                                    c->prm.ros_cap, cat, un, tn, S, n, c->stream));
}

int fire_set_tile(fire_ctx *c, int32_t tile_x, int32_t tile_y) {
    if (!c || !tile_ok(&c->mesh, tile_x, tile_y)) return FIRE_ERR_ARG;
    c->tile_x = tile_x;
    c->tile_y = tile_y;
    return FIRE_OK;
}

int fire_get_tile(fire_ctx *c, int32_t *tile_x, int32_t *tile_y) {
    if (!c || !tile_x || !tile_y) return FIRE_ERR_ARG;
    *tile_x = c->tile_x;
    *tile_y = c->tile_y;
    return FIRE_OK;
}

int fire_set_stream(fire_ctx *c, void *stream) {
    if (!c) return FIRE_ERR_ARG;
    c->stream = (hipStream_t)stream;
    return FIRE_OK;
}

void fire_destroy(fire_ctx *c) {
    if (!c) return;
    for (int i = 0; i < 2; i++)
        if (c->ev[i]) {
            if (c->ev_valid[i]) (void)hipEventSynchronize(c->ev[i]);   // copy into host_status
            (void)hipEventDestroy(c->ev[i]);
        }
    if (c->host_status) (void)hipHostFree(c->host_status);
    delete c;
}

}  // extern "C"
