// C ABI of the batched ensemble: many fire domains of different sizes stepped
// by one kernel launch per time step.  Arena layout, work-list construction,
// device-side model time and the tile autotuner.  The method's arithmetic is
// the same per-tile routine the single-domain kernel runs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fire_internal.h"

using namespace fire;

struct fire_ens {
    int ndom, ncat, dtype, sr_x, sr_y;
    fire_params prm;
    std::vector<fire_mesh> meshes;
    std::vector<int64_t> cell_off, atm_off;   // ndom + 1 entries
    std::vector<int32_t> nign;
    std::vector<fire_ignition> ign_host;      // FIRE_MAX_IGNITIONS slots per member
    char *arena;
    size_t off_coef, off_fuel, off_ign, off_geo, off_cnt, off_dom, off_map, off_status, off_t,
        off_psi[2], off_tign, off_frac, total;
    size_t map_cap;                            // capacity of the tile -> domain map
    const uint8_t *cat;
    const void *dzdx, *dzdy;
    hipStream_t stream;
    int tile_x, tile_y, ntiles;
    int schedule;   // FIRE_ENS_GRID or FIRE_ENS_RESIDENT
    int slots;      // resident work-groups of the current tile shape
};

namespace {

int hip_fail(hipError_t e) { return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP; }

bool ens_meshes_ok(const fire_mesh *m, int ndom) {
    if (!m || ndom < 1 || ndom > 65535) return false;
    for (int k = 0; k < ndom; k++) {
        if (!mesh_ok(&m[k])) return false;
        if (m[k].dtype != m[0].dtype || m[k].sr_x != m[0].sr_x || m[k].sr_y != m[0].sr_y)
            return false;
    }
    return true;
}

void offsets(const fire_mesh *m, int ndom, int64_t *cell, int64_t *atm) {
    cell[0] = atm[0] = 0;
    for (int k = 0; k < ndom; k++) {
        const int64_t nax = (m[k].nx + m[k].sr_x - 1) / m[k].sr_x;
        const int64_t nay = (m[k].ny + m[k].sr_y - 1) / m[k].sr_y;
        cell[k + 1] = cell[k] + (int64_t)m[k].nx * m[k].ny;
        atm[k + 1] = atm[k] + nax * nay;
    }
}

// Arena: per-domain tables first, then the concatenated state arrays.
size_t layout(fire_ens *e) {
    const size_t es = e->dtype == FIRE_F64 ? 8 : 4;
    const size_t ncell = (size_t)e->cell_off[e->ndom];
    size_t o = 0;
    e->off_coef = o;
    o = align_up(o + (size_t)e->ncat * kNCoef * es);
    e->off_fuel = o;
    o = align_up(o + (size_t)e->ncat * sizeof(fire_fuel));
    e->off_ign = o;
    o = align_up(o + (size_t)e->ndom * FIRE_MAX_IGNITIONS * sizeof(fire_ignition));
    e->off_geo = o;
    o = align_up(o + (size_t)e->ndom * kIgnTableBytes);
    e->off_cnt = o;
    o = align_up(o + 8 * sizeof(int32_t));
    e->off_dom = o;
    o = align_up(o + (size_t)e->ndom * sizeof(EnsDomain));
    // the work list is longest for the smallest tile (sr_x x sr_y): one entry
    // per atmosphere cell
    e->map_cap = (size_t)e->atm_off[e->ndom];
    e->off_map = o;
    o = align_up(o + e->map_cap * sizeof(int32_t));
    e->off_status = o;
    o = align_up(o + (size_t)e->ndom * sizeof(int32_t));
    e->off_t = o;
    o = align_up(o + sizeof(EnsClock));
    e->off_psi[0] = o;
    o = align_up(o + ncell * es);
    e->off_psi[1] = o;
    o = align_up(o + ncell * es);
    e->off_tign = o;
    o = align_up(o + ncell * es);
    e->off_frac = o;
    o = align_up(o + ncell * es);
    e->total = o;
    return o;
}

char *ptr(fire_ens *e, size_t off) { return e->arena + off; }

// Domain table and tile -> domain work list for the current tile shape and
// schedule: members in index order on the grid schedule, largest first on
// the resident one (so the bands end with small members' tiles).
int build_worklist(fire_ens *e) {
    std::vector<EnsDomain> doms(e->ndom);
    std::vector<int32_t> map;
    map.reserve(e->map_cap);
    std::vector<int> order(e->ndom);
    for (int k = 0; k < e->ndom; k++) order[k] = k;
    if (e->schedule == FIRE_ENS_RESIDENT)
        std::stable_sort(order.begin(), order.end(), [e](int a, int b) {
            return (int64_t)e->meshes[a].nx * e->meshes[a].ny >
                   (int64_t)e->meshes[b].nx * e->meshes[b].ny;
        });
    int tile0 = 0;
    for (int k : order) {
        const fire_mesh &m = e->meshes[k];
        EnsDomain &d = doms[k];
        std::memset(&d, 0, sizeof(d));
        d.nx = m.nx;
        d.ny = m.ny;
        d.tiles_x = (m.nx + e->tile_x - 1) / e->tile_x;
        const int tiles_y = (m.ny + e->tile_y - 1) / e->tile_y;
        d.tile0 = tile0;
        d.nax = (m.nx + m.sr_x - 1) / m.sr_x;
        d.nay = (m.ny + m.sr_y - 1) / m.sr_y;
        d.nign = e->nign[k];
        d.dx = m.dx;
        d.dy = m.dy;
        d.rdx = 1.0 / m.dx;
        d.rdy = 1.0 / m.dy;
        d.cell_off = e->cell_off[k];
        d.atm_off = e->atm_off[k];
        ignition_window(e->ign_host.data() + (size_t)k * FIRE_MAX_IGNITIONS, e->nign[k],
                        &d.t_ign_lo, &d.t_ign_hi);
        const int nt = d.tiles_x * tiles_y;
        for (int i = 0; i < nt; i++) map.push_back(k);
        tile0 += nt;
    }
    if (map.size() > e->map_cap) return FIRE_ERR_ARG;
    e->ntiles = tile0;
    e->slots = 0;
    if (e->schedule == FIRE_ENS_RESIDENT) {
        e->slots = persist_slots(e->dtype, e->tile_y, e->ncat, (size_t)e->cell_off[e->ndom]);
        if (e->slots < 8) return FIRE_ERR_HIP;
    }
    hipError_t h = hipMemcpyAsync(ptr(e, e->off_dom), doms.data(), doms.size() * sizeof(EnsDomain),
                                  hipMemcpyHostToDevice, e->stream);
    if (h == hipSuccess)
        h = hipMemcpyAsync(ptr(e, e->off_map), map.data(), map.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, e->stream);
    if (h == hipSuccess) h = hipStreamSynchronize(e->stream);
    return hip_fail(h);
}

}  // namespace

extern "C" {

int fire_ens_layout(const fire_mesh *meshes, int32_t ndom, int64_t *cell_off, int64_t *atm_off) {
    if (!ens_meshes_ok(meshes, ndom) || !cell_off || !atm_off) return FIRE_ERR_ARG;
    offsets(meshes, ndom, cell_off, atm_off);
    return FIRE_OK;
}

size_t fire_ens_state_bytes(const fire_mesh *meshes, int32_t ndom, int32_t ncat) {
    if (!ens_meshes_ok(meshes, ndom) || ncat < 1 || ncat > 256) return 0;
    fire_ens e;
    e.ndom = ndom;
    e.ncat = ncat;
    e.dtype = meshes[0].dtype;
    e.cell_off.resize(ndom + 1);
    e.atm_off.resize(ndom + 1);
    offsets(meshes, ndom, e.cell_off.data(), e.atm_off.data());
    return layout(&e);
}

int fire_ens_init(fire_ens **out, const fire_mesh *meshes, int32_t ndom, const fire_fuel *cats,
                  int32_t ncat, const uint8_t *fuel_cat, const void *dzdx, const void *dzdy,
                  const fire_ignition *ign, const int32_t *nign, const fire_params *prm,
                  void *state, size_t state_bytes, void *stream) {
    if (!out) return FIRE_ERR_ARG;
    *out = nullptr;
    if (!ens_meshes_ok(meshes, ndom) || !fuels_ok(cats, ncat) || !fuel_cat || !dzdx || !dzdy ||
        !params_ok(prm) || !state || !nign || ((uintptr_t)state % kAlign) != 0)
        return FIRE_ERR_ARG;
    int64_t total_ign = 0;
    for (int k = 0; k < ndom; k++) {
        if (!ignitions_ok(ign ? ign + total_ign : nullptr, nign[k])) return FIRE_ERR_ARG;
        total_ign += nign[k];
    }
    fire_ens *e = new (std::nothrow) fire_ens();
    if (!e) return FIRE_ERR_OOM;
    e->ndom = ndom;
    e->ncat = ncat;
    e->dtype = meshes[0].dtype;
    e->sr_x = meshes[0].sr_x;
    e->sr_y = meshes[0].sr_y;
    e->prm = *prm;
    e->meshes.assign(meshes, meshes + ndom);
    e->cell_off.resize(ndom + 1);
    e->atm_off.resize(ndom + 1);
    offsets(meshes, ndom, e->cell_off.data(), e->atm_off.data());
    e->nign.assign(nign, nign + ndom);
    e->arena = (char *)state;
    if (state_bytes < layout(e)) {
        delete e;
        return FIRE_ERR_ARG;
    }
    e->cat = fuel_cat;
    e->dzdx = dzdx;
    e->dzdy = dzdy;
    e->stream = (hipStream_t)stream;
    e->schedule = FIRE_ENS_GRID;
    default_tile(&meshes[0], &e->tile_x, &e->tile_y);
    if (!tile_ok(&meshes[0], e->tile_x, e->tile_y)) {
        delete e;
        return FIRE_ERR_ARG;
    }

    // ignition records padded to FIRE_MAX_IGNITIONS per domain
    std::vector<fire_ignition> &igs = e->ign_host;
    igs.assign((size_t)ndom * FIRE_MAX_IGNITIONS, fire_ignition());
    std::memset(igs.data(), 0, igs.size() * sizeof(fire_ignition));
    for (int k = 0, o = 0; k < ndom; o += nign[k], k++)
        for (int g = 0; g < nign[k]; g++) igs[(size_t)k * FIRE_MAX_IGNITIONS + g] = ign[o + g];
    hipError_t h = hipMemcpyAsync(ptr(e, e->off_fuel), cats, sizeof(fire_fuel) * ncat,
                                  hipMemcpyHostToDevice, e->stream);
    if (h == hipSuccess)
        h = hipMemcpyAsync(ptr(e, e->off_ign), igs.data(), igs.size() * sizeof(fire_ignition),
                           hipMemcpyHostToDevice, e->stream);
    const EnsClock clk0 = {prm->t0, 0, 0};
    if (h == hipSuccess)
        h = hipMemcpyAsync(ptr(e, e->off_t), &clk0, sizeof(EnsClock), hipMemcpyHostToDevice,
                           e->stream);
    if (h == hipSuccess) h = hipStreamSynchronize(e->stream);
    if (h == hipSuccess)
        h = launch_coef(e->dtype, (const fire_fuel *)ptr(e, e->off_fuel), ncat, prm->wind_cap,
                        ptr(e, e->off_coef), e->stream);
    if (h == hipSuccess)
        h = hipMemsetAsync(ptr(e, e->off_status), 0, (size_t)ndom * sizeof(int32_t), e->stream);
    const size_t es = e->dtype == FIRE_F64 ? 8 : 4;
    for (int k = 0; k < ndom && h == hipSuccess; k++) {
        const fire_mesh &m = meshes[k];
        double psi0 = prm->psi_init;
        if (!(psi0 > 0.0))
            psi0 = std::sqrt((m.nx * m.dx) * (m.nx * m.dx) + (m.ny * m.dy) * (m.ny * m.dy));
        const size_t o = (size_t)e->cell_off[k] * es;
        h = launch_fill(e->dtype, ptr(e, e->off_psi[0]) + o, ptr(e, e->off_tign) + o,
                        ptr(e, e->off_frac) + o, (size_t)m.nx * m.ny, psi0, e->stream);
    }
    if (h != hipSuccess) {
        delete e;
        return FIRE_ERR_HIP;
    }
    const int rc = build_worklist(e);
    if (rc != FIRE_OK) {
        delete e;
        return rc;
    }
    *out = e;
    return FIRE_OK;
}

int fire_ens_step(fire_ens *e, const void *u, const void *v, double dt, void *flux_sens,
                  void *flux_lat) {
    if (!e || !u || !v || !flux_sens || !flux_lat) return FIRE_ERR_ARG;
    if (!(dt > 0.0) || !std::isfinite(dt)) return FIRE_ERR_ARG;
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tile_x = e->tile_x;
    a.tile_y = e->tile_y;
    a.ntiles = e->ntiles;
    a.per_xcd = (e->ntiles + 7) / 8;
    a.sr_x = e->sr_x;
    a.sr_y = e->sr_y;
    a.ncat = e->ncat;
    a.guard = e->prm.guard_width;
    a.visc_mode = e->prm.viscosity_mode;
    a.dt = dt;
    a.eps = e->prm.viscosity;
    a.ros_cap = e->prm.ros_cap;
    StepBuffers b;
    std::memset(&b, 0, sizeof(b));
    b.psi_in = ptr(e, e->off_psi[0]);     // the clock picks the current one
    b.psi_out = ptr(e, e->off_psi[1]);
    b.tign = ptr(e, e->off_tign);
    b.frac = ptr(e, e->off_frac);
    b.u = u;
    b.v = v;
    b.dzdx = e->dzdx;
    b.dzdy = e->dzdy;
    b.cat = e->cat;
    b.coef = ptr(e, e->off_coef);
    b.fsens = flux_sens;
    b.flat = flux_lat;
    b.status = (int *)ptr(e, e->off_status);
    b.ncells = (size_t)e->cell_off[e->ndom];
    b.ign = (const fire_ignition *)ptr(e, e->off_ign);
    b.ign_tab = ptr(e, e->off_geo);
    b.ndom = e->ndom;
    b.ens_counters = (int32_t *)ptr(e, e->off_cnt);
    b.ens_slots = e->schedule == FIRE_ENS_RESIDENT ? e->slots : 0;
    b.ens_doms = (const EnsDomain *)ptr(e, e->off_dom);
    b.ens_tile_dom = (const int32_t *)ptr(e, e->off_map);
    b.ens_clock = (const EnsClock *)ptr(e, e->off_t);
    hipError_t h = launch_step(e->dtype, a, b, e->stream);
    if (h == hipSuccess) h = launch_advance_clock((EnsClock *)ptr(e, e->off_t), dt, e->stream);
    return h == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

namespace {
int read_clock(fire_ens *e, EnsClock *c) {
    hipError_t h = hipMemcpyAsync(c, ptr(e, e->off_t), sizeof(EnsClock), hipMemcpyDeviceToHost,
                                  e->stream);
    if (h == hipSuccess) h = hipStreamSynchronize(e->stream);
    return hip_fail(h);
}
}  // namespace

int fire_ens_get_state(fire_ens *e, fire_view *out) {
    if (!e || !out) return FIRE_ERR_ARG;
    EnsClock c;
    const int rc = read_clock(e, &c);
    if (rc != FIRE_OK) return rc;
    out->psi = ptr(e, e->off_psi[c.cur ? 1 : 0]);
    out->tign = ptr(e, e->off_tign);
    out->frac = ptr(e, e->off_frac);
    out->t = c.t;
    return FIRE_OK;
}

int fire_ens_status(fire_ens *e, int32_t *status) {
    if (!e || !status) return FIRE_ERR_ARG;
    hipError_t h = hipMemcpyAsync(status, ptr(e, e->off_status), (size_t)e->ndom * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, e->stream);
    if (h == hipSuccess) h = hipStreamSynchronize(e->stream);
    return hip_fail(h);
}

int fire_ens_set_tile(fire_ens *e, int32_t tile_x, int32_t tile_y) {
    if (!e || !tile_ok(&e->meshes[0], tile_x, tile_y)) return FIRE_ERR_ARG;
    e->tile_x = tile_x;
    e->tile_y = tile_y;
    return build_worklist(e);
}

int fire_ens_set_schedule(fire_ens *e, int32_t schedule) {
    if (!e || (schedule != FIRE_ENS_GRID && schedule != FIRE_ENS_RESIDENT)) return FIRE_ERR_ARG;
    const int old = e->schedule;
    e->schedule = schedule;
    const int rc = build_worklist(e);
    if (rc != FIRE_OK) {
        e->schedule = old;
        (void)build_worklist(e);
    }
    return rc;
}

int fire_ens_get_schedule(fire_ens *e, int32_t *schedule) {
    if (!e || !schedule) return FIRE_ERR_ARG;
    *schedule = e->schedule;
    return FIRE_OK;
}

int fire_ens_get_tile(fire_ens *e, int32_t *tile_x, int32_t *tile_y) {
    if (!e || !tile_x || !tile_y) return FIRE_ERR_ARG;
    *tile_x = e->tile_x;
    *tile_y = e->tile_y;
    return FIRE_OK;
}

size_t fire_ens_tune_bytes(fire_ens *e) {
    if (!e) return 0;
    const size_t es = e->dtype == FIRE_F64 ? 8 : 4;
    const size_t n = (size_t)e->cell_off[e->ndom] * es;
    return align_up(n) * 3 + align_up((size_t)e->ndom * sizeof(int32_t)) +
           align_up(sizeof(EnsClock));
}

int fire_ens_autotune(fire_ens *e, const void *u, const void *v, double dt, void *flux_sens,
                      void *flux_lat, const int32_t *cand, int32_t ncand, int32_t reps,
                      void *scratch, size_t scratch_bytes, int32_t *best) {
    if (!e || !cand || ncand < 1 || reps < 1 || !scratch || !best) return FIRE_ERR_ARG;
    if (scratch_bytes < fire_ens_tune_bytes(e) || ((uintptr_t)scratch % kAlign) != 0)
        return FIRE_ERR_ARG;
    for (int i = 0; i < ncand; i++)
        if (!tile_ok(&e->meshes[0], cand[2 * i], cand[2 * i + 1])) return FIRE_ERR_ARG;
    const size_t es = e->dtype == FIRE_F64 ? 8 : 4;
    const size_t n = (size_t)e->cell_off[e->ndom] * es;
    char *sc = (char *)scratch;
    const size_t o_psi = 0, o_tign = align_up(n), o_frac = 2 * align_up(n), o_st = 3 * align_up(n),
                 o_t = o_st + align_up((size_t)e->ndom * sizeof(int32_t));
    // snapshot (psi of the current buffer, t_i, F, status, device clock)
    auto copy = [&](void *dst, const void *src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, e->stream);
    };
    EnsClock clk;
    if (read_clock(e, &clk) != FIRE_OK) return FIRE_ERR_HIP;
    const int cur0 = clk.cur ? 1 : 0;
    hipError_t h = copy(sc + o_psi, ptr(e, e->off_psi[cur0]), n);
    if (h == hipSuccess) h = copy(sc + o_tign, ptr(e, e->off_tign), n);
    if (h == hipSuccess) h = copy(sc + o_frac, ptr(e, e->off_frac), n);
    if (h == hipSuccess) h = copy(sc + o_st, ptr(e, e->off_status), (size_t)e->ndom * 4);
    if (h == hipSuccess) h = copy(sc + o_t, ptr(e, e->off_t), sizeof(EnsClock));
    if (h != hipSuccess) return FIRE_ERR_HIP;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess) {
        if (ev0) (void)hipEventDestroy(ev0);
        return FIRE_ERR_HIP;
    }
    float best_ms = 0.0f;
    int best_i = -1, rc = FIRE_OK;
    for (int i = 0; i < ncand && rc == FIRE_OK; i++) {
        rc = fire_ens_set_tile(e, cand[2 * i], cand[2 * i + 1]);
        if (rc != FIRE_OK) break;
        rc = fire_ens_step(e, u, v, dt, flux_sens, flux_lat);   // warm-up
        if (rc != FIRE_OK) break;
        (void)hipEventRecord(ev0, e->stream);
        for (int r = 0; r < reps && rc == FIRE_OK; r++)
            rc = fire_ens_step(e, u, v, dt, flux_sens, flux_lat);
        (void)hipEventRecord(ev1, e->stream);
        if (hipEventSynchronize(ev1) != hipSuccess) rc = FIRE_ERR_HIP;
        float ms = 0.0f;
        if (rc == FIRE_OK && hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess) rc = FIRE_ERR_HIP;
        if (rc == FIRE_OK && (best_i < 0 || ms < best_ms)) {
            best_ms = ms;
            best_i = i;
        }
        // restore the snapshot into the buffer that is current again
        h = copy(ptr(e, e->off_psi[cur0]), sc + o_psi, n);
        if (h == hipSuccess) h = copy(ptr(e, e->off_tign), sc + o_tign, n);
        if (h == hipSuccess) h = copy(ptr(e, e->off_frac), sc + o_frac, n);
        if (h == hipSuccess) h = copy(ptr(e, e->off_status), sc + o_st, (size_t)e->ndom * 4);
        if (h == hipSuccess) h = copy(ptr(e, e->off_t), sc + o_t, sizeof(EnsClock));
        if (h != hipSuccess) rc = FIRE_ERR_HIP;
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (rc != FIRE_OK) return rc;
    best[0] = cand[2 * best_i];
    best[1] = cand[2 * best_i + 1];
    rc = fire_ens_set_tile(e, best[0], best[1]);
    if (rc == FIRE_OK && hipStreamSynchronize(e->stream) != hipSuccess) rc = FIRE_ERR_HIP;
    return rc;
}

int fire_ens_set_stream(fire_ens *e, void *stream) {
    if (!e) return FIRE_ERR_ARG;
    e->stream = (hipStream_t)stream;
    return FIRE_OK;
}

void fire_ens_destroy(fire_ens *e) { delete e; }

}  // extern "C"
