// Coupling input of the fire step (Sect. 6): the atmosphere's staggered
// horizontal wind brought to the centres of the fire cells.
//
// 1. k_wind_vertical, one thread per staggered point (u-points at the
//    x-faces, v-points at the y-faces of the atmospheric cells, Fig. 1):
//    heights of the cell centres above the terrain from the geopotential,
//    z_k = (phi_k + phi_{k+1}) / 2g - h, averaged over the two columns that
//    share the face (the one column at the domain edge), and the value at
//    z_f from the piecewise-linear interpolant in ln z through (ln z0, 0)
//    and the level values above z0 (0 if z_f <= z0, the top value above the
//    highest level).  Computed in double (float logarithms for float
//    arrays, see ln_z).
// 2. k_wind_bilinear, 8 fire rows per work-group: bilinear interpolation
//    of each component from its staggered points, coordinates clamped to
//    the points' extent, in the array precision -- first in y, once per
//    point of the row's span (into LDS), then in x per fire cell.  The kernel
//    writes 2 values per fire cell and reads fields ~sr_x sr_y times smaller,
//    so it is bound by the HBM writes.
#include <cmath>
#include <mutex>

#include "fire_internal.h"

// Scratch of the no-allocation entry point fire_wind_interp_static: the two
// staggered surface fields, one copy on each GPU for the life of the
// process.  Host code never uses this name as an address; it uses the
// pointer hipGetSymbolAddress returns for the current device
// (static_scratch()).
static __device__ __align__(256) char scratch[FIRE_WIND_STATIC_BYTES];

namespace fire {
namespace {

constexpr int kWB = 256;

struct WindArgs {
    int32_t nax, nay, nz, sr_x, sr_y, nx, ny;
    int32_t vec;       // rows of 4k cells and 4-element-aligned outputs: vector stores
    double zf, g;
    double lzf;        // ln z_f
    double rsx, rsy;   // 1 / sr_x, 1 / sr_y
};

// ln z of a height formed in double.  For a float result the logarithm is
// taken in float (the hardware base-2 logarithm times ln 2: a few ulp,
// ~1e-7 of the interpolation weights, far below the float rounding of the
// result); heights stay in double, since they are differences of large
// geopotential heights.  Double arrays take the double logarithm.
template <typename T> __device__ __forceinline__ double ln_z(double z);
template <> __device__ __forceinline__ double ln_z<float>(double z) {
    return (double)(__builtin_amdgcn_logf((float)z) * 0.693147180559945309f);
}
template <> __device__ __forceinline__ double ln_z<double>(double z) { return ::log(z); }

template <typename T>
__device__ __forceinline__ double cell_z(const T *phi, const T *hgt, int ncol, int k, int c,
                                         double g) {
    return 0.5 * ((double)phi[(size_t)k * ncol + c] + (double)phi[(size_t)(k + 1) * ncol + c]) / g -
           (double)hgt[c];
}

template <typename T>
__global__ void __launch_bounds__(kWB)
k_wind_vertical(const WindArgs a, const T *u3, const T *v3, const T *phi, const T *hgt,
                const T *z0, T *uf, T *vf) {
    const int nu = (a.nax + 1) * a.nay, nv = a.nax * (a.nay + 1);
    const int idx = blockIdx.x * kWB + threadIdx.x;
    if (idx >= nu + nv) return;
    const int ncol = a.nax * a.nay;
    int ca, cb, np, pi;
    const T *val;
    if (idx < nu) {   // u-point (I, J) on the x-face between columns I-1 and I
        const int J = idx / (a.nax + 1), I = idx - J * (a.nax + 1);
        ca = J * a.nax + (I > 0 ? I - 1 : 0);
        cb = J * a.nax + (I < a.nax ? I : a.nax - 1);
        val = u3;
        np = nu;
        pi = idx;
    } else {          // v-point (I, J) on the y-face between rows J-1 and J
        const int q = idx - nu;
        const int J = q / a.nax, I = q - J * a.nax;
        ca = (J > 0 ? J - 1 : 0) * a.nax + I;
        cb = (J < a.nay ? J : a.nay - 1) * a.nax + I;
        val = v3;
        np = nv;
        pi = q;
    }
    const double zr = 0.5 * ((double)z0[ca] + (double)z0[cb]);
    double r = 0.0;
    if (a.zf > zr) {
        const double lzf = a.lzf;
        double lz_prev = ln_z<T>(zr), v_prev = 0.0;
        bool done = false;
        for (int k = 0; k < a.nz && !done; k++) {
            const double zk = 0.5 * (cell_z(phi, hgt, ncol, k, ca, a.g) +
                                     cell_z(phi, hgt, ncol, k, cb, a.g));
            if (!(zk > zr)) continue;
            const double vk = (double)val[(size_t)k * np + pi];
            const double lzk = ln_z<T>(zk);
            if (lzf <= lzk) {
                r = v_prev + (lzf - lz_prev) * ((vk - v_prev) / (lzk - lz_prev));
                done = true;
            } else {
                lz_prev = lzk;
                v_prev = vk;
            }
        }
        if (!done) r = v_prev;
    }
    if (idx < nu) uf[pi] = T(r);
    else vf[pi] = T(r);
}

// Interpolation position along one axis of a point field of n points at
// coordinate p = N / Dn (an exact rational: fire centres and face points sit
// at multiples of 1/(2 sr) in atmosphere-cell units), clamped to [0, n - 1]:
// lower point k0, upper k1, weight t (exact up to one rounding of rem/Dn).
template <typename T> struct Axis {
    int k0, k1;
    T t;
};

template <typename T> __device__ __forceinline__ Axis<T> axis(int N, int Dn, T rDn, int n) {
    Axis<T> r;
    if (n == 1) {
        r.k0 = r.k1 = 0;
        r.t = T(0);
    } else if (N <= 0) {
        r.k0 = 0;
        r.k1 = 1;
        r.t = T(0);
    } else if (N >= (n - 1) * Dn) {
        r.k0 = n - 2;
        r.k1 = n - 1;
        r.t = T(1);
    } else {
        // N / Dn from the reciprocal, then corrected to the exact quotient
        int k = (int)((float)N * (float)rDn);
        int rem = N - k * Dn;
        if (rem < 0) {
            k--;
            rem += Dn;
        } else if (rem >= Dn) {
            k++;
            rem -= Dn;
        }
        r.k0 = k;
        r.k1 = k + 1;
        r.t = T(rem) * rDn;
    }
    return r;
}

// A work-group takes kWChunk consecutive cells of kWRows consecutive fire
// rows.  Per row the y-interpolation is done once per staggered point the
// chunk spans, into a line in LDS (the y weights are the same along the row;
// two lines alternate, so one barrier per row suffices); each thread then
// interpolates its 4 consecutive cells in x from that line, with the x
// positions and weights formed once for all the rows, and, when rows are
// 4-aligned, stores them as one 16-byte non-temporal vector.  A fire centre
// is at x/DX = (i + 1/2)/sr_x; u-points at (I, J + 1/2), v-points at
// (I + 1/2, J) in atmosphere-cell units.  Arithmetic in the array precision.
constexpr int kWChunk = 4 * kWB;
constexpr int kWRows = 8;
// staggered points a chunk can span: (kWChunk - 1)/sr_x + 3 at most
constexpr int kWLine = kWChunk + 4;

template <typename T> using W4 = T __attribute__((ext_vector_type(4)));

template <typename T>
__global__ void __launch_bounds__(kWB)
k_wind_bilinear(const WindArgs a, const T *uf, const T *vf, T *u, T *v) {
    __shared__ T Lu[2][kWLine], Lv[2][kWLine];
    // row bands along x (up to 2^21 of them), chunks along y (up to 2^14)
    const int j0 = blockIdx.x * kWRows;
    const int c0 = blockIdx.y * kWChunk;
    const int Dx = 2 * a.sr_x, Dy = 2 * a.sr_y;
    const T rx = T(a.rsx) * T(0.5), ry = T(a.rsy) * T(0.5);
    // x/DX = (2i + 1) / (2 sr_x), shifted by -1/2 (= -sr_x / (2 sr_x)) for v;
    // point ranges [ub, ue], [vb, ve] of the chunk's cells
    const int c1 = (c0 + kWChunk < a.nx ? c0 + kWChunk : a.nx) - 1;
    const int ub = axis(2 * c0 + 1, Dx, rx, a.nax + 1).k0;
    const int ue = axis(2 * c1 + 1, Dx, rx, a.nax + 1).k1;
    const int vb = axis(2 * c0 + 1 - a.sr_x, Dx, rx, a.nax).k0;
    const int ve = axis(2 * c1 + 1 - a.sr_x, Dx, rx, a.nax).k1;
    // this thread's cells: line positions and weights, the same in every row
    const int i0 = c0 + 4 * threadIdx.x;
    int uk0[4], uk1[4], vk0[4], vk1[4];
    T ut[4], vt[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int i = i0 + q < a.nx ? i0 + q : a.nx - 1;
        const Axis<T> ux = axis(2 * i + 1, Dx, rx, a.nax + 1);
        const Axis<T> vx = axis(2 * i + 1 - a.sr_x, Dx, rx, a.nax);
        uk0[q] = ux.k0 - ub;
        uk1[q] = ux.k1 - ub;
        ut[q] = ux.t;
        vk0[q] = vx.k0 - vb;
        vk1[q] = vx.k1 - vb;
        vt[q] = vx.t;
    }
    const bool vec = a.vec != 0;
    const int j1 = j0 + kWRows < a.ny ? j0 + kWRows : a.ny;
    int p = 0;
    for (int j = j0; j < j1; j++, p ^= 1) {
        const Axis<T> uy = axis(2 * j + 1 - a.sr_y, Dy, ry, a.nay);
        const Axis<T> vy = axis(2 * j + 1, Dy, ry, a.nay + 1);
        const T *u0 = uf + (size_t)uy.k0 * (a.nax + 1), *u1 = uf + (size_t)uy.k1 * (a.nax + 1);
        const T *v0 = vf + (size_t)vy.k0 * a.nax, *v1 = vf + (size_t)vy.k1 * a.nax;
        // (line p was last read in row j - 2, before every thread reached the
        // barrier of row j - 1)
        for (int q = threadIdx.x; q <= ue - ub && q < kWLine; q += kWB)
            Lu[p][q] = (T(1) - uy.t) * u0[ub + q] + uy.t * u1[ub + q];
        for (int q = threadIdx.x; q <= ve - vb && q < kWLine; q += kWB)
            Lv[p][q] = (T(1) - vy.t) * v0[vb + q] + vy.t * v1[vb + q];
        __syncthreads();
        if (i0 < a.nx) {
            T ou[4], ov[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                ou[q] = (T(1) - ut[q]) * Lu[p][uk0[q]] + ut[q] * Lu[p][uk1[q]];
                ov[q] = (T(1) - vt[q]) * Lv[p][vk0[q]] + vt[q] * Lv[p][vk1[q]];
            }
            const size_t row = (size_t)j * a.nx;
            if (vec) {   // streaming (non-temporal) stores: the output is not re-read here
                const W4<T> wu = {ou[0], ou[1], ou[2], ou[3]}, wv = {ov[0], ov[1], ov[2], ov[3]};
                __builtin_nontemporal_store(wu, reinterpret_cast<W4<T> *>(u + row + i0));
                __builtin_nontemporal_store(wv, reinterpret_cast<W4<T> *>(v + row + i0));
            } else {
                for (int q = 0; q < 4 && i0 + q < a.nx; q++) {
                    u[row + i0 + q] = ou[q];
                    v[row + i0 + q] = ov[q];
                }
            }
        }
    }
}

bool grid_ok(const fire_wind_grid *g) {
    if (!g) return false;
    if (g->nax < 1 || g->nay < 1 || g->nz < 1 || g->sr_x < 1 || g->sr_y < 1) return false;
    if (g->nx < 1 || g->ny < 1 || g->nx > (int64_t)g->nax * g->sr_x ||
        g->ny > (int64_t)g->nay * g->sr_y)
        return false;
    if ((int64_t)g->nx * g->ny > ((int64_t)1 << 31)) return false;
    if (g->nx >= (1 << 24) || g->ny >= (1 << 24)) return false;   // axis positions in int/float
    if ((int64_t)(g->nax + 1) * (g->nay + 1) * 2 > ((int64_t)1 << 31)) return false;
    if (!(g->zf > 0.0) || !std::isfinite(g->zf) || !(g->g > 0.0) || !std::isfinite(g->g))
        return false;
    return g->dtype == FIRE_F32 || g->dtype == FIRE_F64;
}

size_t stag_elems(const fire_wind_grid *g) {
    return (size_t)(g->nax + 1) * g->nay + (size_t)g->nax * (g->nay + 1);
}

template <typename T>
hipError_t run(const fire_wind_grid *g, const void *u3, const void *v3, const void *phi,
               const void *hgt, const void *z0, void *u, void *v, void *scratch,
               hipStream_t s) {
    WindArgs a;
    a.nax = g->nax;
    a.nay = g->nay;
    a.nz = g->nz;
    a.sr_x = g->sr_x;
    a.sr_y = g->sr_y;
    a.nx = g->nx;
    a.ny = g->ny;
    a.vec = (g->nx % 4 == 0) && ((uintptr_t)u % (4 * sizeof(T)) == 0) &&
            ((uintptr_t)v % (4 * sizeof(T)) == 0);
    a.zf = g->zf;
    a.g = g->g;
    a.lzf = std::log(g->zf);
    a.rsx = 1.0 / g->sr_x;   // 1/(2 sr) = rs / 2 is exact in binary
    a.rsy = 1.0 / g->sr_y;
    T *uf = (T *)scratch;
    T *vf = uf + (size_t)(g->nax + 1) * g->nay;
    const int npts = (int)stag_elems(g);
    hipLaunchKernelGGL(k_wind_vertical<T>, dim3((npts + kWB - 1) / kWB), dim3(kWB), 0, s, a,
                       (const T *)u3, (const T *)v3, (const T *)phi, (const T *)hgt,
                       (const T *)z0, uf, vf);
    hipLaunchKernelGGL(k_wind_bilinear<T>,
                       dim3((g->ny + kWRows - 1) / kWRows, (g->nx + kWChunk - 1) / kWChunk),
                       dim3(kWB), 0, s, a, (const T *)uf, (const T *)vf, (T *)u, (T *)v);
    return hipGetLastError();
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per
// device; nullptr on failure.
void *static_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace fire

using namespace fire;

extern "C" {

size_t fire_wind_scratch_bytes(const fire_wind_grid *g) {
    if (!grid_ok(g)) return 0;
    return align_up(stag_elems(g) * (g->dtype == FIRE_F64 ? 8 : 4));
}

int fire_wind_interp(const fire_wind_grid *g, const void *u3, const void *v3, const void *phi,
                     const void *hgt, const void *z0, void *u, void *v, void *scratch,
                     size_t scratch_bytes, void *stream) {
    if (!grid_ok(g) || !u3 || !v3 || !phi || !hgt || !z0 || !u || !v || !scratch)
        return FIRE_ERR_ARG;
    if (scratch_bytes < fire_wind_scratch_bytes(g) || ((uintptr_t)scratch % kAlign) != 0)
        return FIRE_ERR_ARG;
    const hipError_t h =
        g->dtype == FIRE_F64
            ? run<double>(g, u3, v3, phi, hgt, z0, u, v, scratch, (hipStream_t)stream)
            : run<float>(g, u3, v3, phi, hgt, z0, u, v, scratch, (hipStream_t)stream);
    return h == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

int fire_wind_interp_static(const fire_wind_grid *g, const void *u3, const void *v3,
                            const void *phi, const void *hgt, const void *z0, void *u, void *v,
                            void *stream) {
    if (!grid_ok(g) || !u3 || !v3 || !phi || !hgt || !z0 || !u || !v) return FIRE_ERR_ARG;
    if (fire_wind_scratch_bytes(g) > (size_t)FIRE_WIND_STATIC_BYTES) return FIRE_ERR_TOO_LARGE;
    void *buf = static_scratch();   // device address of `scratch` on this GPU
    if (!buf) return FIRE_ERR_HIP;
    const hipError_t h =
        g->dtype == FIRE_F64
            ? run<double>(g, u3, v3, phi, hgt, z0, u, v, buf, (hipStream_t)stream)
            : run<float>(g, u3, v3, phi, hgt, z0, u, v, buf, (hipStream_t)stream);
    return h == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

}  // extern "C"
