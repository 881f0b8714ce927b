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

struct StepArgs {
    int32_t nx, ny;
    int32_t tile_x, tile_y;
    int32_t tiles_x, ntiles, per_xcd;
    int32_t sr_x, sr_y, nax, nay;
    int32_t ncat, guard, visc_mode, nign, pad;
    double dx, dy;
    double rdx, rdy;     // 1/dx, 1/dy
    double t, dt;
    double eps, ros_cap;
    fire_ignition ign[FIRE_MAX_IGNITIONS];
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
};

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

}  // namespace fire
