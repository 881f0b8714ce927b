/*
 * fire.h -- C ABI of the MI355X (gfx950) fire-mesh time step.
 *
 * The method is the fire module of WRF-Fire as described by Mandel, Beezley
 * & Kochanski, "Coupled atmosphere-wildland fire modeling with WRF-Fire
 * version 3.3" (arXiv:1102.1343).  One call of fire_step() makes one time
 * step of the fire model in the order of Sect. 6:
 *   1. ignition of active segment / drip-torch ignitions (Sect. 4.4,
 *      Eqs. 20-21),
 *   2. Heun step (Eq. 11) of the level-set equation (Eq. 10) with the
 *      upwinded, viscous right-hand side of Eqs. (12)-(13), the spread rate
 *      of Eq. (3) evaluated from the normal wind and slope, and the boundary
 *      extrapolation of Sect. 4.1,
 *   3. ignition times of nodes crossed during the step (Eq. 14),
 *   4. fuel fraction by the sub-cell quadrature of Eqs. (15)-(19),
 *   5. sensible and latent heat flux densities (Eqs. 5-6),
 *   6. their mean over the fire cells of each atmosphere cell (Sect. 6),
 * plus the boundary check of Sect. 4.1 (fire near the boundary ends the run).
 *
 * All per-cell arrays are device memory, row-major [ny][nx] with x fastest,
 * cell (i, j) centred at ((i + 1/2) dx, (j + 1/2) dy).  Floating arrays have
 * the element type chosen by fire_mesh.dtype (float or double).  Atmosphere
 * arrays are [ceil(ny/sr_y)][ceil(nx/sr_x)].
 *
 * Ownership: the caller owns every device buffer -- inputs, the state arena
 * and the outputs.  The library owns only the context (host memory) and
 * allocates no device memory.  Every call is asynchronous on the context's
 * stream unless stated otherwise; no function throws.
 *
 * Errors: functions return FIRE_OK (0) or a negative FIRE_ERR_* code;
 * fire_strerror() names it.  Argument errors are detected before anything is
 * enqueued.  Errors of earlier asynchronous work surface as FIRE_ERR_HIP from
 * a later call.
 */
#ifndef FIRE_H
#define FIRE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FIRE_ABI_VERSION 3

enum {
    FIRE_OK = 0,
    FIRE_ERR_ARG = -1,       /* invalid argument (size, pointer, value)      */
    FIRE_ERR_HIP = -2,       /* a HIP runtime call or kernel launch failed   */
    FIRE_ERR_OOM = -3,       /* host allocation of the context failed        */
    FIRE_ERR_BOUNDARY = -4,  /* fire reached the guard ring (Sect. 4.1)      */
    FIRE_ERR_NONFINITE = -5, /* non-finite level set or fuel fraction        */
    FIRE_ERR_STATE = -6,     /* call not allowed in the context's state      */
    FIRE_ERR_TOO_LARGE = -7  /* input larger than a fixed-size buffer allows */
};

/* sticky status bits reported by fire_status() */
enum { FIRE_STATUS_BOUNDARY = 1, FIRE_STATUS_NONFINITE = 2 };

typedef enum { FIRE_F32 = 0, FIRE_F64 = 1 } fire_dtype;

/* Fire mesh (Sect. 3): nx x ny cells of dx x dy metres; sr_x x sr_y fire
 * cells make one atmosphere cell (refinement ratio, Sect. 8.3).  Needs
 * nx, ny >= 2, 1 <= sr_x <= 122, 1 <= sr_y <= 26. */
typedef struct {
    int32_t nx, ny;
    double dx, dy;
    int32_t sr_x, sr_y;
    int32_t dtype;            /* fire_dtype */
    int32_t reserved;
} fire_mesh;

/* One fuel category: the quantities of Table 1 in SI units. */
typedef struct {
    double windrf;            /* a, wind reduction from 6.1 m to midflame     */
    double tf;                /* T_f (s); if <= 0, T_f = -600 w/(1000 ln 0.6) */
    double weight;            /* w (s), used only when tf <= 0 (Eq. 4)        */
    double fgi;               /* w_l total fuel load (kg/m^2)                 */
    double fueldepthm;        /* delta (m)                                    */
    double savr;              /* sigma, surface/volume ratio (1/m)            */
    double fuelmce;           /* M_x, moisture of extinction                  */
    double fueldens;          /* rho_P, oven-dry particle density (kg/m^3)    */
    double st;                /* S_T, total mineral content                   */
    double se;                /* S_E, effective mineral content               */
    double cmbcnst;           /* h, heat content of dry fuel (J/kg)           */
    double fuelmc_g;          /* M_f, fuel moisture content                   */
    double ros_mult;          /* per-category spread multiplier m_k (1)       */
    int32_t ichap;            /* non-zero: chaparral spread rate, Eq. (2)     */
    int32_t reserved;
} fire_fuel;

/* Ignition (Sect. 4.4).  Segment a-b (a point when a == b) started at t_start
 * with initial spread rate ros until the distance radius is reached; with
 * (vx, vy) != 0 a drip torch starting at a with velocity v until t_end
 * (b unused).  ros = +inf ignites the disc of the given radius at once, in
 * the step that starts exactly at t_start. */
typedef struct {
    double ax, ay, bx, by;    /* m                                            */
    double t_start;           /* t_g (s)                                      */
    double radius;            /* r_g (m)                                      */
    double ros;               /* S_g (m/s)                                    */
    double vx, vy;            /* drip-torch velocity (m/s)                    */
    double t_end;             /* t_h (s)                                      */
} fire_ignition;

#define FIRE_MAX_IGNITIONS 8

typedef struct {
    double viscosity;         /* epsilon of Eq. (12), 0.4 in the paper        */
    double psi_init;          /* initial level set (> 0); <= 0: domain diagonal */
    double wind_cap;          /* e of Eq. (3) for Rothermel fuels (30 m/s)    */
    double ros_cap;           /* upper cap on S (m/s); +inf for none          */
    double t0;                /* initial time (s)                             */
    int32_t guard_width;      /* guard ring width (cells) of the boundary check */
    int32_t boundary_policy;  /* 0: stop at fire in the guard ring, 1: continue */
    int32_t viscosity_mode;   /* 0: eps*S*Lap~ psi; 1: eps*Lap~ psi (literal) */
    int32_t reserved;
} fire_params;

typedef struct fire_ctx fire_ctx;

/* Device pointers into the state arena and the model time. */
typedef struct {
    const void *psi;          /* level set psi [ny][nx]                       */
    const void *tign;         /* ignition time t_i [ny][nx], +inf = not yet   */
    const void *frac;         /* fuel fraction F [ny][nx]                     */
    double t;                 /* model time of this state (s)                 */
} fire_view;

/* Bytes of caller-owned device memory the state arena needs for this mesh
 * and number of fuel categories (psi double buffer, t_i, F, coefficient
 * table, status word, and the step's ignition set-up: a 4-byte word and 8
 * bounds per tile of the default tile shape and 16 offsets per mesh row,
 * ntiles (4 + 8 e) + 16 (ny + 48) e bytes for element size e).  Returns 0
 * for an invalid mesh. */
size_t fire_state_bytes(const fire_mesh *mesh, int32_t ncat);

/*
 * Create a context and initialise the state (Sect. 4.4): psi = psi_init,
 * t_i = +inf, F = 1, time t0.  The per-category spread-rate coefficients of
 * Eqs. (1)-(3) / Table 2, the burn time of Eq. (4) and the flux factors of
 * Eqs. (5)-(6) are computed on the device into the arena.
 *   mesh, cats[ncat], ign[nign], prm : host structs, copied
 *   fuel_cat : device uint8 [ny][nx], values < ncat (checked by the caller)
 *   dzdx, dzdy : device [ny][nx] terrain gradient (Sect. 6, preprocessing)
 *   state : device arena of at least fire_state_bytes(), 256-byte aligned
 *   stream : hipStream_t (NULL = default stream)
 * fuel_cat, dzdx, dzdy and state must stay valid until fire_destroy().
 * 1 <= ncat <= 256, 0 <= nign <= FIRE_MAX_IGNITIONS.
 */
int fire_init(fire_ctx **out, const fire_mesh *mesh, const fire_fuel *cats, int32_t ncat,
              const uint8_t *fuel_cat, const void *dzdx, const void *dzdy,
              const fire_ignition *ign, int32_t nign, const fire_params *prm,
              void *state, size_t state_bytes, void *stream);

/*
 * One fire time step of length dt (> 0) driven by the surface wind (u, v)
 * (device [ny][nx], m/s at 6.1 m, on fire cell centres).  Writes the mean
 * sensible and latent heat flux densities (W/m^2) over the step into
 * flux_sens / flux_lat (device atmosphere arrays) and updates the state in
 * the arena.  If out is not NULL it receives device pointers to the new
 * psi, t_i and F (valid until the next fire_step) and the new time.  Enqueues
 * the fused step kernel and, while an ignition is active (Sect. 4.4), a small
 * kernel before it that forms the step's ignition geometry and per-tile
 * set-up in the arena.
 *
 * Boundary policy 0 (Sect. 4.1: the run terminates when fire reaches the
 * guard ring): after each step the status word is copied to pinned host
 * memory on the stream, and each call reads the copies of earlier steps
 * before enqueueing its own -- the copy of the step before the last is
 * waited for (so the host runs at most one step ahead of what it has
 * checked), the last one only if it has already completed.  When a copy
 * shows fire in the guard ring the call enqueues nothing and returns
 * FIRE_ERR_BOUNDARY, or FIRE_ERR_NONFINITE for a non-finite psi or F; every
 * later call returns the same code without stepping.  The state then holds
 * the step that set the bit or at most one step more; fire_status() (which
 * waits) reports the bits exactly and also stops the run.  With policy 1
 * nothing waits and the conditions are only recorded in the status word.
 */
int fire_step(fire_ctx *ctx, const void *u, const void *v, double dt, void *flux_sens,
              void *flux_lat, fire_view *out);

/* Current state pointers and time (no copy). */
int fire_get_state(fire_ctx *ctx, fire_view *out);

/* Replace the state by device copies of psi, t_i and F (each [ny][nx]) and
 * set the time (checkpoint restore).  The status word is cleared. */
int fire_set_state(fire_ctx *ctx, const void *psi, const void *tign, const void *frac, double t);

/* Waits for the context's stream and returns the sticky FIRE_STATUS_* bits
 * (>= 0), or a negative error code.  Under boundary policy 0 a set bit also
 * stops later fire_step() calls. */
int fire_status(fire_ctx *ctx);

/* The tile shape fire_init() picks for this mesh (host only, no device
 * call): the widest multiple of sr_x up to 122 columns and the tallest
 * multiple of sr_y up to 20 rows (sr_y itself when sr_y > 20), within the
 * limits of fire_set_tile().  FIRE_ERR_ARG for an invalid mesh. */
int fire_default_tile(const fire_mesh *mesh, int32_t *tile_x, int32_t *tile_y);

/* Copies the per-category coefficient table to host memory (waits):
 * out[ncat][10] as doubles, columns S0 R0 b c d e m T_f C_h C_q. */
int fire_coef(fire_ctx *ctx, double *out, int32_t ncat);

/* Spread rate of Eq. (3) for n points (test entry): S[k] from category
 * cat[k], normal wind un[k] and normal slope tn[k] (device arrays of the
 * context dtype).  Asynchronous. */
int fire_ros_eval(fire_ctx *ctx, const uint8_t *cat, const void *un, const void *tn, void *S,
                  int64_t n);

/* Tile shape of the fused step kernel: tile_x a multiple of sr_x with
 * tile_x <= 122, tile_y a multiple of sr_y with tile_y <= 42 (FP32) or
 * <= 26 (FP64).  Results do not depend on the tile shape.  The arena holds
 * the per-tile ignition set-up for as many tiles as the default shape has;
 * with a smaller tile the tiles past that count evaluate every active
 * ignition at every node (same results, slower while ignitions are
 * active). */
int fire_set_tile(fire_ctx *ctx, int32_t tile_x, int32_t tile_y);
int fire_get_tile(fire_ctx *ctx, int32_t *tile_x, int32_t *tile_y);

/* Change the stream later calls enqueue on. */
int fire_set_stream(fire_ctx *ctx, void *stream);

const char *fire_strerror(int code);
int fire_abi_version(void);

/* Releases the context (no device memory is freed: the caller owns it). */
void fire_destroy(fire_ctx *ctx);

/* ------------------------------------------------------------------------
 * Ensemble: many independent fire domains of different sizes advanced by one
 * kernel launch per step (the data-parallel use that ensemble data
 * assimilation makes of the model, Sect. 11.5: many fire simulations, each
 * the method of fire_step() unchanged).  Every member
 * computes exactly what a single-domain context with the same mesh, fuels,
 * ignitions and parameters computes, bit for bit, whatever the tile shape.
 *
 * Members share the fuel table, the parameters, dtype and the refinement
 * ratio; they differ in nx, ny, dx, dy, terrain, wind and ignitions.  Per-cell
 * arrays of all members are concatenated: member k's [ny_k][nx_k] block starts
 * at element cell_off[k]; atmosphere arrays likewise at atm_off[k]
 * (fire_ens_layout()).  The model time and the index of the current psi
 * buffer live on the device (advanced by a one-thread kernel after each step),
 * so fire_ens_step() enqueues the same three kernels every call (the step's
 * ignition geometry, the step, the clock) and may be captured once in a HIP
 * graph and replayed: each replay is one step.
 *
 * Two schedules of the step kernel, with the same results bit for bit:
 *   FIRE_ENS_GRID     one work-group per tile of the members' work list
 *                     (members in index order);
 *   FIRE_ENS_RESIDENT as many work-groups as fit on the device at once, each
 *                     taking tiles from a counter over its band of the work
 *                     list, members ordered largest first.
 * ---------------------------------------------------------------------- */
typedef struct fire_ens fire_ens;

#define FIRE_ENS_GRID 0
#define FIRE_ENS_RESIDENT 1

/* Element offsets of the members' blocks: cell_off[ndom + 1] into per-cell
 * arrays and atm_off[ndom + 1] into atmosphere arrays (host arrays written by
 * the call; the last entry is the total).  All meshes must be valid and share
 * dtype, sr_x and sr_y; 1 <= ndom <= 65535. */
int fire_ens_layout(const fire_mesh *meshes, int32_t ndom, int64_t *cell_off, int64_t *atm_off);

/* Bytes of the caller-owned device arena for the ensemble (0 if invalid). */
size_t fire_ens_state_bytes(const fire_mesh *meshes, int32_t ndom, int32_t ncat);

/*
 * Create an ensemble and initialise every member as fire_init() does.
 *   meshes[ndom], cats[ncat], prm : host, copied
 *   fuel_cat, dzdx, dzdy : device, concatenated per-cell arrays
 *   ign : host, the members' ignitions one after another, nign[k] of member
 *         k (0 <= nign[k] <= FIRE_MAX_IGNITIONS); NULL if all are 0
 *   state : device arena of fire_ens_state_bytes(), 256-byte aligned
 * Waits for the set-up copies; fuel_cat, dzdx, dzdy and state must stay
 * valid until fire_ens_destroy().
 */
int fire_ens_init(fire_ens **out, const fire_mesh *meshes, int32_t ndom, const fire_fuel *cats,
                  int32_t ncat, const uint8_t *fuel_cat, const void *dzdx, const void *dzdy,
                  const fire_ignition *ign, const int32_t *nign, const fire_params *prm,
                  void *state, size_t state_bytes, void *stream);

/* One step of length dt of every member, winds u, v as concatenated per-cell
 * arrays, fluxes into concatenated atmosphere arrays.  Never waits; the
 * boundary condition of a member only sets its status bits (boundary policy
 * 1 for all members).  Enqueues three kernels and nothing else. */
int fire_ens_step(fire_ens *e, const void *u, const void *v, double dt, void *flux_sens,
                  void *flux_lat);

/* Device pointers to the concatenated psi, t_i, F and the model time (waits
 * for the stream to read the device-side time). */
int fire_ens_get_state(fire_ens *e, fire_view *out);

/* Sticky FIRE_STATUS_* bits of every member into host status[ndom] (waits). */
int fire_ens_status(fire_ens *e, int32_t *status);

/* Tile shape (same limits as fire_set_tile()); rebuilds the tile work list
 * (waits).  Not to be called during graph capture. */
int fire_ens_set_tile(fire_ens *e, int32_t tile_x, int32_t tile_y);
int fire_ens_get_tile(fire_ens *e, int32_t *tile_x, int32_t *tile_y);

/* Schedule of the step kernel (FIRE_ENS_GRID, the default, or
 * FIRE_ENS_RESIDENT); rebuilds the work list (waits).  FIRE_ERR_ARG for any
 * other value; FIRE_ERR_HIP if the device's occupancy cannot be queried (the
 * schedule is then unchanged).  Not to be called during graph capture. */
int fire_ens_set_schedule(fire_ens *e, int32_t schedule);
int fire_ens_get_schedule(fire_ens *e, int32_t *schedule);

/* Device scratch bytes fire_ens_autotune() needs (a snapshot of the state). */
size_t fire_ens_tune_bytes(fire_ens *e);

/*
 * Times reps steps for each candidate tile shape cand[2*i], cand[2*i+1]
 * (i < ncand) with the given inputs, keeps the fastest (written to best[2])
 * and restores the state, time and status from a snapshot in the caller's
 * scratch (fire_ens_tune_bytes(), 256-byte aligned), so the ensemble is left
 * as before the call except for the tile shape.  The flux buffers are
 * overwritten.  Waits.
 */
int fire_ens_autotune(fire_ens *e, const void *u, const void *v, double dt, void *flux_sens,
                      void *flux_lat, const int32_t *cand, int32_t ncand, int32_t reps,
                      void *scratch, size_t scratch_bytes, int32_t *best);

int fire_ens_set_stream(fire_ens *e, void *stream);

/* Releases the ensemble handle (host memory only). */
void fire_ens_destroy(fire_ens *e);

/* ------------------------------------------------------------------------
 * Adjoint (reverse mode) of a run of fire steps.  A differentiable run
 * advances a context nsteps steps of length dt under one surface wind
 * (u, v), keeping psi every `every` steps; the backward pass takes dL/dF
 * of the fuel fraction after the last step and returns
 *   dL/du, dL/dv   per cell, summed over the steps;
 *   dL/dm_k        per fuel category, m_k the spread multiplier
 *                  (fire_fuel.ros_mult, Eq. 3);
 *   dL/d(shift)    per ignition, the translation of its start point and
 *                  segment (the centre of a point ignition, Sect. 4.4).
 * Derivatives are those of the discrete step along the branches the forward
 * took (Godunov side, spread-rate clamps and cap, ghost formula, ignition
 * minimum, crossing step of Eq. 14, signs in Eqs. 15-19).  Results do not
 * depend on `every` (segments are replayed bit for bit).
 * ---------------------------------------------------------------------- */
typedef struct fire_adj fire_adj;

/* Bytes of caller-owned device scratch for a differentiable run of nsteps
 * steps with a checkpoint every `every` steps: about
 * (nsteps/every + 6 every + 26) x nx x ny elements (two sets of replay
 * buffers, so one segment is replayed while the next is reversed).  0 if
 * invalid. */
size_t fire_adj_bytes(const fire_mesh *mesh, int32_t ncat, int32_t nsteps, int32_t every);

/* Attach to a context (which must outlive the handle); scratch is device
 * memory of fire_adj_bytes(), 256-byte aligned.  Creates one stream (default
 * priority) and five events for the backward pass; FIRE_ERR_HIP if that
 * fails. */
int fire_adj_init(fire_adj **out, fire_ctx *ctx, int32_t nsteps, int32_t every, void *scratch,
                  size_t scratch_bytes);

/* Run the context nsteps steps from its current state with wind u, v
 * (device [ny][nx], kept by pointer until the backward pass) and step dt,
 * recording what the backward pass needs.  The context ends after the last
 * step; F there is the run's output.  Returns fire_step's errors. */
int fire_adj_forward(fire_adj *a, const void *u, const void *v, double dt);

/* Backward pass for dF = dL/dF_end (device [ny][nx]): writes grad_u, grad_v
 * (device [ny][nx], context dtype), grad_mult (host double[ncat]) and, if not
 * NULL, grad_shift (host double[2 nign], x then y per ignition).  The context
 * must not have been stepped since fire_adj_forward (FIRE_ERR_STATE).
 * Segment replays run on the handle's own stream, ordered by events against
 * the context's stream, which does the rest.  Waits for both. */
int fire_adj_backward(fire_adj *a, const void *dF, void *grad_u, void *grad_v,
                      double *grad_mult, double *grad_shift);

/* Releases the handle, its stream and events (waits for its stream). */
void fire_adj_destroy(fire_adj *a);

/* ------------------------------------------------------------------------
 * Coupling input (Sect. 6): the atmosphere's staggered horizontal wind to
 * the fire cell centres.  The atmosphere mesh has nax x nay cells of
 * (sr_x dx) x (sr_y dy) covering the fire mesh from the same corner, and nz
 * cells in the vertical.  u lives on the x-faces (nax + 1 per row), v on
 * the y-faces (nay + 1 per column), Fig. 1.  For each face point the wind at
 * height zf above the terrain is the piecewise-linear interpolant in ln z
 * through (ln z0, 0) and the level values at the heights of the cell
 * centres, z_k = (phi_k + phi_{k+1}) / (2 g) - hgt, taken from the two
 * columns sharing the face (averaged; the one column at the domain edge);
 * levels at or below z0 are left out, the top value is kept above the
 * highest level, and zf <= z0 gives 0.  Each component is then
 * interpolated bilinearly to the fire cell centres, coordinates clamped to
 * the extent of its face points.  The result is the (u, v) fire_step takes.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t nax, nay, nz;     /* atmosphere cells in x and y; vertical cells  */
    int32_t sr_x, sr_y;       /* fire cells per atmosphere cell              */
    int32_t nx, ny;           /* fire mesh, nx <= nax sr_x, ny <= nay sr_y,
                                 both < 2^24, nx ny <= 2^31                   */
    int32_t dtype;            /* fire_dtype of every array                   */
    double zf;                /* height of the fire wind above terrain (m), 6.1 */
    double g;                 /* gravitational acceleration (m/s^2), 9.81    */
} fire_wind_grid;

/* Bytes of device scratch fire_wind_interp needs (0 if the grid is invalid). */
size_t fire_wind_scratch_bytes(const fire_wind_grid *grid);

/*
 * Device arrays, row-major with x fastest:
 *   u3  [nz][nay][nax+1]   u on the x-faces (m/s)
 *   v3  [nz][nay+1][nax]   v on the y-faces (m/s)
 *   phi [nz+1][nay][nax]   geopotential at the cell bottoms/tops (m^2/s^2)
 *   hgt [nay][nax]         terrain height (m)
 *   z0  [nay][nax]         roughness height (m)
 *   u, v [ny][nx]          output, wind at zf on the fire cell centres
 * scratch: device, fire_wind_scratch_bytes(), 256-byte aligned.
 * Asynchronous on stream.
 */
int fire_wind_interp(const fire_wind_grid *grid, const void *u3, const void *v3,
                     const void *phi, const void *hgt, const void *z0, void *u, void *v,
                     void *scratch, size_t scratch_bytes, void *stream);

/* Size of the library's own scratch for fire_wind_interp_static (16 MiB on
 * each GPU it runs on, held until the process ends). */
#define FIRE_WIND_STATIC_BYTES (16u << 20)

/*
 * fire_wind_interp() for callers that cannot allocate device memory (code
 * under HIP-graph capture, serving loops, harnesses that forbid allocation):
 * the same computation and results, bit for bit, with the scratch taken from
 * a fixed buffer inside the library instead of the caller.  Nothing is
 * allocated.  The caller still passes the inputs and the outputs u, v.
 * Returns FIRE_ERR_TOO_LARGE when fire_wind_scratch_bytes(grid) exceeds
 * FIRE_WIND_STATIC_BYTES (about 2 million staggered points in FP32, half that
 * in FP64; an 820 x 820 atmosphere needs 5.4 MB in FP32).  Every call on one
 * GPU uses the same buffer: calls that overlap in time on one GPU (different
 * streams, or threads without ordering) race and give undefined results;
 * calls on one stream are ordered and safe.  Asynchronous on stream.
 */
int fire_wind_interp_static(const fire_wind_grid *grid, const void *u3, const void *v3,
                            const void *phi, const void *hgt, const void *z0, void *u, void *v,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FIRE_H */
