// HIP kernels (gfx950, wave64) of the WRF-Fire fire-mesh time step
// (Mandel, Beezley & Kochanski, arXiv:1102.1343).
//
// k_step is the whole step fused into one pass over the mesh: a work-group
// loads its tile plus three halo rings into LDS once, applies the ignitions
// (Sect. 4.4), runs both Heun stages of the level-set equation (Eqs. 10-13)
// with the boundary extrapolation of Sect. 4.1 redone for each stage, sets
// the ignition times (Eq. 14), integrates the fuel fraction over sub-cells
// (Eqs. 15-19), forms the heat fluxes (Eqs. 5-6) and averages them over the
// atmosphere cells of the tile (Sect. 6).  Tiles are multiples of the
// refinement ratio, so every atmosphere cell is reduced inside one
// work-group in a fixed order: no atomics, bitwise reproducible.
//
// HBM traffic per cell and step is one read of psi, t_i, F, u, v, dz/dx,
// dz/dy, category and one write of psi and F (t_i only where it changes);
// halo re-reads come from L2.  Work-groups are remapped so that each of the
// eight XCDs sweeps a contiguous band of tiles, keeping halo rows in its L2.
#include "fire_device.h"

namespace fire {
namespace {

using namespace dev;

// Right-hand side of Eq. (12) at frame cell (fy, fx) of the level set P.
template <typename T, typename RowPtr>
__device__ __forceinline__ T rhs(const T (*P)[kFW], int fy, int fx, T u, T v, T gzx, T gzy,
                                 RowPtr row, const Consts<T> &c) {
    return rhs5(P[fy][fx], P[fy][fx - 1], P[fy][fx + 1], P[fy - 1][fx], P[fy + 1][fx], u, v, gzx,
                gzy, row, c);
}

// Global loads/stores at element index i.  With SMALL (every array below
// 4 GiB) the byte offset is formed in 32 bits, which lets the compiler use
// scalar-base addressing with a 32-bit vector offset.
template <bool SMALL, typename T> __device__ __forceinline__ const T &at(const T *p, uint32_t i) {
    if (SMALL)
        return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) +
                                            i * (uint32_t)sizeof(T));
    return p[i];
}
template <bool SMALL, typename T> __device__ __forceinline__ T &at(T *p, uint32_t i) {
    if (SMALL)
        return *reinterpret_cast<T *>(reinterpret_cast<char *>(p) + i * (uint32_t)sizeof(T));
    return p[i];
}

// Per-cell inputs of the right-hand side: category, wind, terrain gradient.
template <typename T> struct Inputs {
    T u, v, gx, gy;
    int cv;
};

template <bool SMALL, typename T>
__device__ __forceinline__ Inputs<T> load_inputs(uint32_t idx, const uint8_t *cat, const T *uw,
                                                 const T *vw, const T *dzdx, const T *dzdy) {
    Inputs<T> r;
    r.cv = at<SMALL>(cat, idx);
    r.u = at<SMALL>(uw, idx);
    r.v = at<SMALL>(vw, idx);
    r.gx = at<SMALL>(dzdx, idx);
    r.gy = at<SMALL>(dzdy, idx);
    return r;
}

// Fill the one-cell ghost ring of frame P around the domain (Sect. 4.1).
// Ghost nodes read in-domain nodes only, so the ring fills in one pass.
// Corners (x and y outside) are the x extrapolation of the ghost row.
template <typename T>
__device__ __forceinline__ void ghost_node(T (*P)[kFW], int fy, int fx, int gx, int gy, int nx,
                                           int ny, bool corners) {
    const bool xin = gx >= 0 && gx < nx, yin = gy >= 0 && gy < ny;
    const int sx = gx == -1 ? 1 : (gx == nx ? -1 : 0);
    const int sy = gy == -1 ? 1 : (gy == ny ? -1 : 0);
    if (yin && sx != 0) {
        P[fy][fx] = ghost(P[fy][fx + sx], P[fy][fx + 2 * sx]);
    } else if (xin && sy != 0) {
        P[fy][fx] = ghost(P[fy + sy][fx], P[fy + 2 * sy][fx]);
    } else if (corners && sx != 0 && sy != 0) {
        const T r1 = ghost(P[fy + sy][fx + sx], P[fy + 2 * sy][fx + sx]);
        const T r2 = ghost(P[fy + sy][fx + 2 * sx], P[fy + 2 * sy][fx + 2 * sx]);
        P[fy][fx] = ghost(r1, r2);
    }
}

// A copy of a wave-uniform value that the compiler cannot see through.  The
// step takes one per phase for the frame-row bounds, so the per-row range
// masks formed from them are not shared between phases (held across the
// kernel, they would be spilled and reloaded row by row).
__device__ __forceinline__ int phase_copy(int v) {
    asm volatile("" : "+s"(v));
    return v;
}

// Lane permutations within each row of 16 lanes (DPP): swap neighbours,
// swap pairs, mirror each half row, mirror the row.  A lane whose source is
// unavailable keeps its own value.
template <int CTRL> __device__ __forceinline__ float dpp(float x) {
    const int i = __builtin_bit_cast(int, x);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(i, i, CTRL, 0xf, 0xf, false));
}
template <int CTRL> __device__ __forceinline__ double dpp(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
    const uint32_t l2 = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
    const uint32_t h2 = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)h2 << 32) | l2);
}
__device__ __forceinline__ float lane_value(float x, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}
__device__ __forceinline__ double lane_value(double x, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Largest value over the wave's 64 lanes (NaN ignored, as by vmax), the same
// in every lane: the maximum of each 16-lane row by four lane permutations,
// then of the four rows.  The wave must have every lane active.
template <typename T> __device__ __forceinline__ T wave_reduce_max(T m) {
    m = vmax(m, dpp<0xB1>(m));    // quad_perm [1, 0, 3, 2]
    m = vmax(m, dpp<0x4E>(m));    // quad_perm [2, 3, 0, 1]
    m = vmax(m, dpp<0x141>(m));   // row_half_mirror
    m = vmax(m, dpp<0x140>(m));   // row_mirror
    return vmax(vmax(lane_value(m, 0), lane_value(m, 16)),
                vmax(lane_value(m, 32), lane_value(m, 48)));
}

// Bounds of psi_g (Eq. 21) over the nodes of a frame of kFW columns and fh
// rows whose first node is global (fx0, fy0): the distance from the frame's
// centre to the segment -/+ the frame's half diagonal, less the radius,
// widened by a margin (1 m + 1e-4 of the distances) far above the rounding of
// psi_g and of the bounds themselves.  Node (i, j) sits at ((i + 1/2) dx,
// (j + 1/2) dy), so the centre is (fx0 + kFW/2, fy0 + fh/2) cells.
template <typename T>
__device__ __forceinline__ void ign_frame_bounds(const IgnGeo<T> &gs, int fx0, int fy0, int fh,
                                                 double dx, double dy, T &lb, T &ub) {
    const T cx = T((fx0 + 0.5 * kFW) * dx - gs.ax);
    const T cy = T((fy0 + 0.5 * fh) * dy - gs.ay);
    const T hx = T(0.5 * (kFW - 1)) * T(dx), hy = T(0.5 * (fh - 1)) * T(dy);
    const T hd = M<T>::sqrt(hx * hx + hy * hy);
    const T sp = med3(cx * gs.exL + cy * gs.eyL, T(0), T(1));
    const T qx = cx - sp * gs.ex, qy = cy - sp * gs.ey;
    const T d = M<T>::sqrt(qx * qx + qy * qy);
    const T mg = T(1) + T(1e-4) * (d + M<T>::sqrt(gs.ex * gs.ex + gs.ey * gs.ey));
    lb = d - hd - gs.rad - mg;
    ub = d + hd - gs.rad + mg;
}

// Fuel fraction of one cell at t' (Eqs. 15-19) from the 3x3 node values of
// psi^{n+1} (A) and of the node ignition times t^ (Q, already t' where
// psi >= 0).  Four sub-cells with corners at the centre, two edge midpoints
// and a cell corner, bilinear values, t^ reset to t' where psi >= 0 there.
template <typename T>
__device__ __forceinline__ T cell_fraction(const T (*A)[kFW], int fy, const T (*Q)[kFW], int qy,
                                           int fx, T tp, T rTf) {
    T p[3][3], q[3][3];
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            p[b][a] = A[fy + b - 1][fx + a - 1];
            q[b][a] = Q[qy + b - 1][fx + a - 1];
        }
    // edge midpoints and corners shared by neighbouring sub-cells
    const T pc = p[1][1], qc = q[1][1];
    T pmax = p[0][0];
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
        for (int a = 0; a < 3; a++) pmax = vmax(pmax, p[b][a]);
    // every node burning: every sub-cell corner value is a mean of negative
    // values, so beta = 1 exactly in all four sub-cells (Eq. 18) and t^ is
    // t_i at every corner; the sums keep the general path's order
    const bool all_burning = pmax < T(0);
    T pe[2][2], qe[2][2];   // [0][s]: x edges (s = left/right), [1][s]: y edges
#pragma unroll
    for (int s = 0; s < 2; s++) {
        pe[0][s] = T(0.5) * (pc + p[1][2 * s]);
        qe[0][s] = T(0.5) * (qc + q[1][2 * s]);
        pe[1][s] = T(0.5) * (pc + p[2 * s][1]);
        qe[1][s] = T(0.5) * (qc + q[2 * s][1]);
    }
    T burned = T(0);
#pragma unroll
    for (int sb = 0; sb < 2; sb++)
#pragma unroll
        for (int sa = 0; sa < 2; sa++) {
            const T pk[4] = {pc, pe[0][sa], pe[1][sb],
                             T(0.25) * (pc + p[1][2 * sa] + p[2 * sb][1] + p[2 * sb][2 * sa])};
            const T qk[4] = {qc, qe[0][sa], qe[1][sb],
                             T(0.25) * (qc + q[1][2 * sa] + q[2 * sb][1] + q[2 * sb][2 * sa])};
            if (all_burning) {
                T tau = T(0);
#pragma unroll
                for (int k = 0; k < 4; k++) tau += tp - qk[k];
                burned += M<T>::one_m_exp_neg(T(0.25) * tau * rTf);
                continue;
            }
            T sum = T(0), asum = T(0), tau = T(0);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                sum += pk[k];
                asum += vabs(pk[k]);
                tau += pk[k] >= T(0) ? T(0) : (tp - qk[k]);
            }
            const T beta = asum > T(0) ? T(0.5) * (T(1) - M<T>::div(sum, asum)) : T(0);
            burned += beta * M<T>::one_m_exp_neg(T(0.25) * tau * rTf);
        }
    return T(1) - T(0.25) * burned;
}

// The fused step.  KR = frame rows per thread (frame height <= 4 KR).
// LDS frames: A holds psi^n, then psi^{n+1}, then the latent flux; B holds
// psi*, then the sensible flux; C holds the node ignition times t^.  Each
// frame keeps only the rows it is used on: A all 4 KR, B frame rows
// [1, 4 KR - 1) (row fy at B[fy - 1]), C rows [2, 4 KR - 2) (at C[fy - 2]).
// At the default FP32 tile the plain step then needs under 40 KiB, so four
// work-groups fit in a CU's 160 KiB.
// PRE: the per-tile ignition set-up comes from iuse / ilb / irow (a single
// domain's step); otherwise it is formed here from the geometry table.
template <typename T, int KR, bool SMALL, bool REC, bool PRE>
__device__ __forceinline__ void
step_tile(const StepArgs &a, const int tile, const int tx, const int ty, const uint32_t cbase,
          const double tnow,
          const IgnTable<T> *itab, const T *__restrict__ psi_in, T *__restrict__ psi_out, T *tign, T *frac,
          const T *__restrict__ uw, const T *__restrict__ vw, const T *__restrict__ dzdx,
          const T *__restrict__ dzdy, const uint8_t *__restrict__ cat, const T *__restrict__ coef,
          T *__restrict__ fsens, T *__restrict__ flat, int *status, T *rec_p0, T *rec_b,
          int32_t *mark, const uint32_t *__restrict__ iuse, const T *__restrict__ ilb,
          const T *__restrict__ irow) {
    constexpr int FHM = kNR * KR;
    __shared__ T A[FHM][kFW];
    __shared__ T B[FHM - 2][kFW];
    __shared__ T C[FHM - 4][kFW];
    extern __shared__ __attribute__((aligned(32))) double dyn_smem[];
    T *tab = reinterpret_cast<T *>(dyn_smem);
    // the same table through an LDS pointer: 32-bit row addresses
    const lds_t<T> *tab3 = (const lds_t<T> *)tab;

    const int tyi = tile / a.tiles_x;
    const int txi = tile - tyi * a.tiles_x;
    const int x0 = txi * a.tile_x, y0 = tyi * a.tile_y;
    const int tid = ty * kFW + tx;
    const int nx = a.nx, ny = a.ny;
    const int FH = a.tile_y + 2 * kHalo;
    const int gx = x0 - kHalo + tx;
    const bool colin = gx >= 0 && gx < nx;
    const bool xr1 = colin && tx >= 1 && tx < a.tile_x + 5;
    const bool xr2 = colin && tx >= 2 && tx < a.tile_x + 4;
    const bool xr3 = colin && tx >= 3 && tx < a.tile_x + 3;
    // in-domain frame rows [ylo, yhi)
    const int ylo = kHalo - y0 > 0 ? kHalo - y0 : 0;
    const int yhi = ny - y0 + kHalo < FH ? ny - y0 + kHalo : FH;
    // the in-domain rows of Heun stages 1 and 2 and of the fuel fraction:
    // one range test per row and phase (no range masks shared between
    // phases, which the compiler would keep for the whole kernel)
    const int lo1 = max(1, ylo), hi1 = min(a.tile_y + 5, yhi);
    const int lo2 = max(2, ylo), hi2 = min(a.tile_y + 4, yhi);
    const int lo3 = max(3, ylo), hi3 = min(a.tile_y + 3, yhi);
    // a frame that lies inside the domain has no ghost nodes
    const bool interior = x0 >= kHalo && x0 + a.tile_x + kHalo <= nx && ylo == 0 && yhi == FH;
    // element index of frame row 0 (mod 2^32), plus the domain's first
    // element cbase when the arrays are concatenated; in-domain indices are
    // below 2^32 (2^31 for one domain)
    const uint32_t off0 = cbase + (uint32_t)((y0 - kHalo) * nx + gx);
    const uint32_t unx = (uint32_t)nx;
    // element index of this thread's frame row ty, and the stride between
    // its rows (row k of the thread is fy = ty + kNR k): idx0 + k rstep, so
    // the per-row multiply is uniform (scalar) work
    const uint32_t idx0 = off0 + (uint32_t)ty * unx;
    const uint32_t rstep = __builtin_amdgcn_readfirstlane((uint32_t)kNR * unx);
    // (k rstep is formed where it is used: held in scalar registers for the
    // whole kernel, the seven offsets do not fit the scalar budget of four
    // work-groups per CU)
    auto roff = [&](int k) { return (uint32_t)k * rstep; };

    for (int i = tid; i < a.ncat; i += kBlock)
        make_row(coef + i * kNCoef, tab + i * kLRow, T(a.ros_cap));

    Consts<T> c;
    c.rdx = T(a.rdx);
    c.rdy = T(a.rdy);
    c.eps = T(a.eps);
    c.cap = T(a.ros_cap);
    c.visc_mode = a.visc_mode;
    const T dt = T(a.dt);
    const T hdt = T(0.5 * a.dt);
    const T rdt = T(1.0 / a.dt);
    const T t = T(tnow);
    const T tp = T(tnow + a.dt);
    const T INF = M<T>::inf();
    const uint32_t ncm1 = (uint32_t)(a.ncat - 1);

    // ---- load psi^n on the whole frame and step 1, ignition (Sect. 4.4):
    // psi := min(psi, psi_g); a node lit by this step's ignitions gets the
    // earliest arrival among the ignitions that cover it
    T tig[KR];
    T p0[KR];
#pragma unroll
    for (int k = 0; k < KR; k++) {
        const int fy = ty + kNR * k;
        const bool in = colin && fy >= ylo && fy < yhi;
        p0[k] = in ? at<SMALL>(psi_in, idx0 + roff(k)) : T(0);
        tig[k] = INF;
    }
    if (PRE && a.nign > 0) {
        // the tile's set-up, formed ahead of the step (IgnSetLayout): how
        // each ignition enters the tile and a lower bound of its psi_g there;
        // the row offsets py, by of the wave's frame rows.  No barrier: an
        // ignition that can only lower psi is skipped by a wave whose
        // largest psi^n (NaN nodes, which no ignition changes, ignored) is no
        // larger than that bound.
        T m = -INF;
#pragma unroll
        for (int k = 0; k < KR; k++) m = vmax(m, p0[k]);
        m = wave_reduce_max(m);
        const uint32_t word = iuse[tile < a.tile_cap ? tile : a.tile_cap];
        // a wave's 64 lanes share one frame row
        const int tyu = __builtin_amdgcn_readfirstlane(ty);
        T pold[KR];
#pragma unroll
        for (int k = 0; k < KR; k++) pold[k] = p0[k];
        for (int g = 0; g < a.nign; g++) {
            const int use = (word >> (2 * g)) & 3;
            if (!use) continue;
            // (use 1 occurs only for tiles below the capacity)
            if (use == 1 && ilb[(size_t)tile * FIRE_MAX_IGNITIONS + g] >= m) continue;
            const IgnGeo<T> geo = itab->g[g];
            const T px = ign_px(geo, gx, a.dx);
            // global row gy = y0 - kHalo + fy is table row y0 + fy
            const T *rpy = irow + (size_t)g * a.ign_rows + y0 + tyu;
            const T *rby = irow + (size_t)(FIRE_MAX_IGNITIONS + g) * a.ign_rows + y0 + tyu;
            if (use == 2) {
#pragma unroll
                for (int k = 0; k < KR; k++) ign_apply(geo, px, rpy[kNR * k], rby[kNR * k], p0[k], tig[k]);
            } else {
#pragma unroll
                for (int k = 0; k < KR; k++) ign_lower(geo, px, rpy[kNR * k], rby[kNR * k], p0[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < KR; k++)
            if (!(pold[k] > T(0) && p0[k] <= T(0))) tig[k] = INF;
    } else if (a.nign > 0) {
        // the step's geometry of each ignition (lane g of the first wave
        // takes ignition g) and its per-row offsets py, by for the frame
        // rows, shared through LDS
        __shared__ IgnGeo<T> geo_s[FIRE_MAX_IGNITIONS];
        __shared__ int geo_on[FIRE_MAX_IGNITIONS];
        __shared__ int geo_use[FIRE_MAX_IGNITIONS];   // 0 skip, 1 far, 2 near
        __shared__ T geo_lb[FIRE_MAX_IGNITIONS], geo_ub[FIRE_MAX_IGNITIONS];
        __shared__ T wave_max[kBlock / 64];
        __shared__ T row_py[FIRE_MAX_IGNITIONS][FHM];
        __shared__ T row_by[FIRE_MAX_IGNITIONS][FHM];
        if (tid < a.nign) {
            const IgnGeo<T> gs = itab->g[tid];
            const bool on = itab->on[tid] != 0;
            geo_on[tid] = on ? 1 : 0;
            geo_s[tid] = gs;
            if (on)
                ign_frame_bounds(gs, x0 - kHalo, y0 - kHalo, FHM, a.dx, a.dy, geo_lb[tid],
                                 geo_ub[tid]);
        }
        // the frame's largest psi^n (NaN nodes, which no ignition changes,
        // are ignored): an ignition whose psi_g is provably positive and no
        // smaller than that on every frame node changes nothing here
        T m = -INF;
#pragma unroll
        for (int k = 0; k < KR; k++) m = vmax(m, p0[k]);
        m = wave_reduce_max(m);
        if ((tid & 63) == 0) wave_max[tid >> 6] = m;
        __syncthreads();
        for (int e = tid; e < a.nign * FHM; e += kBlock) {
            const int g = e / FHM, j = e - g * FHM;
            if (geo_on[g]) {
                const T py = ign_py(geo_s[g], y0 - kHalo + j, a.dy);
                row_py[g][j] = py;
                row_by[g][j] = ign_by(geo_s[g], py);
            }
        }
        if (tid < a.nign) {
            int use = geo_on[tid] ? 2 : 0;
            const T lb = geo_lb[tid];
            if (use && lb > T(0)) {
                // psi_g > 0 on every frame node: no node is lit by it.  It
                // is never the minimum either when no smaller than the
                // frame's largest psi^n, or above another active ignition's
                // psi_g everywhere
                use = 1;
                T M = wave_max[0];
                for (int w = 1; w < kBlock / 64; w++) M = vmax(M, wave_max[w]);
                if (lb >= M) use = 0;
                for (int h = 0; h < a.nign; h++)
                    if (h != tid && geo_on[h] && geo_ub[h] < lb) use = 0;
            }
            geo_use[tid] = use;
        }
        __syncthreads();
        T pold[KR];
#pragma unroll
        for (int k = 0; k < KR; k++) pold[k] = p0[k];
        for (int g = 0; g < a.nign; g++) {
            const int use = geo_use[g];
            if (!use) continue;
            const IgnGeo<T> geo = geo_s[g];
            const T px = ign_px(geo, gx, a.dx);
            if (use == 2) {
#pragma unroll
                for (int k = 0; k < KR; k++) {
                    const int fy = ty + kNR * k;
                    ign_apply(geo, px, row_py[g][fy], row_by[g][fy], p0[k], tig[k]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < KR; k++) {
                    const int fy = ty + kNR * k;
                    ign_lower(geo, px, row_py[g][fy], row_by[g][fy], p0[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < KR; k++)
            if (!(pold[k] > T(0) && p0[k] <= T(0))) tig[k] = INF;
    }
    {
        const int fh = phase_copy(FH);
#pragma unroll
        for (int k = 0; k < KR; k++) {
            const int fy = ty + kNR * k;
            if (fy < fh) A[fy][tx] = p0[k];
        }
    }
    __syncthreads();
    if (!interior) {
        const int fh = phase_copy(FH);
#pragma unroll
        for (int k = 0; k < KR; k++) {
            const int fy = ty + kNR * k;
            if (fy < fh) ghost_node(A, fy, tx, gx, y0 - kHalo + fy, nx, ny, false);
        }
        __syncthreads();
    }

    // ---- step 2a: first Heun stage on the tile plus two rings,
    // psi* = psi^n + dt F(psi^n)
    // the per-cell inputs of row k + 1 are loaded while row k computes
    // (rows outside the stage load the domain's first cell instead, unused:
    // unconditional loads need no register copies)
    auto in1 = [&](int k) {
        const int fy = ty + kNR * k;
        return xr1 && fy >= lo1 && fy < hi1;
    };
    auto src1 = [&](int k) { return in1(k) ? idx0 + roff(k) : cbase; };
    Inputs<T> nxt = load_inputs<SMALL>(src1(0), cat, uw, vw, dzdx, dzdy);
#pragma unroll
    for (int k = 0; k < KR; k++) {
        const int fy = ty + kNR * k;
        const Inputs<T> cur = nxt;
        if (k + 1 < KR) nxt = load_inputs<SMALL>(src1(k + 1), cat, uw, vw, dzdx, dzdy);
        if (in1(k)) {
            const lds_t<T> *row = tab3 + __umul24(min((uint32_t)cur.cv, ncm1), (uint32_t)kLRow);
            const T F1 = rhs(A, fy, tx, cur.u, cur.v, cur.gx, cur.gy, row, c);
            B[fy - 1][tx] = p0[k] + dt * F1;
        }
    }
    __syncthreads();
    if (!interior) {
        const int fhb = phase_copy(FH - 1);
#pragma unroll
        for (int k = 0; k < KR; k++) {
            const int fy = ty + kNR * k;
            if (fy >= 1 && fy < fhb)
                ghost_node(B, fy - 1, tx, gx, y0 - kHalo + fy, nx, ny, false);
        }
        __syncthreads();
    }

    // ---- step 2b: second stage on the tile plus one ring,
    // psi^{n+1} = (psi^n + psi* + dt F(psi*))/2, Eq. (11); step 3: ignition
    // time of nodes crossed during the step (Eq. 14), first crossing kept;
    // node times t^ = t' where psi^{n+1} >= 0, else t_i (Eq. 17)
    int st = 0;
    const int gw = a.guard;
    auto in2 = [&](int k) {
        const int fy = ty + kNR * k;
        return xr2 && fy >= lo2 && fy < hi2;
    };
    auto src2 = [&](int k) { return in2(k) ? idx0 + roff(k) : cbase; };
    nxt = load_inputs<SMALL>(src2(0), cat, uw, vw, dzdx, dzdy);
#pragma unroll
    for (int k = 0; k < KR; k++) {
        const int fy = ty + kNR * k;
        const Inputs<T> cur = nxt;
        if (k + 1 < KR) nxt = load_inputs<SMALL>(src2(k + 1), cat, uw, vw, dzdx, dzdy);
        if (in2(k)) {
            const int gy = y0 - kHalo + fy;
            const uint32_t idx = idx0 + roff(k);
            const lds_t<T> *row = tab3 + __umul24(min((uint32_t)cur.cv, ncm1), (uint32_t)kLRow);
            const T F2 = rhs(B, fy - 1, tx, cur.u, cur.v, cur.gx, cur.gy, row, c);
            const T pn0 = A[fy][tx];
            const T pn = T(0.5) * (pn0 + B[fy - 1][tx]) + hdt * F2;
            A[fy][tx] = pn;   // stage-1 reads of A ended at the last barrier
            // t_i is read only where it can matter: a burning node, a node
            // crossing zero, or a node lit by this step's ignition
            T ti = INF, told = INF;
            if (!REC && (pn <= T(0) || tig[k] < INF)) {
                told = at<SMALL>(tign, idx);
                ti = told;
                if (is_inf(ti)) ti = tig[k];
                if (pn0 > T(0) && pn <= T(0) && is_inf(ti))
                    ti = t + M<T>::div(pn0 * dt, pn0 - pn);
            }
            if (!REC) C[fy - 2][tx] = pn >= T(0) ? tp : ti;
            if (xr3 && fy >= 3 && fy < a.tile_y + 3) {
                at<SMALL>(psi_out, idx) = pn;
                if (REC) {   // psi' and psi* of the step, for the reverse pass
                    at<SMALL>(rec_p0, idx) = pn0;
                    at<SMALL>(rec_b, idx) = B[fy - 1][tx];
                } else {
                    if (!(ti == told)) {
                        at<SMALL>(tign, idx) = ti;
                        // the step in which t_i was first set
                        if (mark && is_inf(told)) at<SMALL>(mark, idx) = a.mark_step;
                    }
                    const bool edge = gx < gw || gy < gw || gx >= nx - gw || gy >= ny - gw;
                    if (edge && pn < T(0)) st |= kStBoundary;
                    if (!__builtin_isfinite(pn)) st |= kStNonfinite;
                }
            }
        }
    }
    // a replay for the reverse pass needs psi only: no fuel fraction or flux
    if (REC) return;
    __syncthreads();
    if (!interior) {
        // ghost psi re-extrapolated, corners included; ghost t^ = t' (R19)
        const int fh = phase_copy(FH);
#pragma unroll
        for (int k = 0; k < KR; k++) {
            const int fy = ty + kNR * k;
            const int gy = y0 - kHalo + fy;
            if (fy < fh) {
                ghost_node(A, fy, tx, gx, gy, nx, ny, true);
                if (!(colin && gy >= 0 && gy < ny) && fy >= 2 && fy < fh - 2)
                    C[fy - 2][tx] = tp;
            }
        }
        __syncthreads();
    }

    // ---- steps 4-5: fuel fraction at t' (Eqs. 15-19) and cell fluxes
    // (Eqs. 5-6).  A cell whose nine stencil nodes all have psi >= 0 has no
    // burning sub-cell point: beta = 0 in every sub-cell and F = 1 exactly.
    // The sensible flux goes straight to B (not read in this phase).
    T fl[KR];
    auto in3 = [&](int k) {
        const int fy = ty + kNR * k;
        return xr3 && fy >= lo3 && fy < hi3;
    };
    // F of row k + 1 is loaded while row k computes
    auto src3 = [&](int k) { return in3(k) ? idx0 + roff(k) : cbase; };
    T fo_next = at<SMALL>(frac, src3(0));
#pragma unroll
    for (int k = 0; k < KR; k++) {
        const int fy = ty + kNR * k;
        T fs = T(0);
        fl[k] = T(0);
        const T fo = fo_next;
        if (k + 1 < KR) fo_next = at<SMALL>(frac, src3(k + 1));
        if (in3(k)) {
            const uint32_t idx = idx0 + roff(k);
            T mn = vmin(vmin(A[fy - 1][tx - 1], A[fy - 1][tx]), A[fy - 1][tx + 1]);
            mn = vmin(mn, vmin(vmin(A[fy][tx - 1], A[fy][tx]), A[fy][tx + 1]));
            mn = vmin(mn, vmin(vmin(A[fy + 1][tx - 1], A[fy + 1][tx]), A[fy + 1][tx + 1]));
            // F^{n+1} = F^n = 1 and no flux unless a stencil node burns or F
            // was already below 1
            if (mn < T(0) || !(fo == T(1))) {
                const int cv = at<SMALL>(cat, idx);
                const lds_t<T> *row = tab3 + __umul24(min((uint32_t)cv, ncm1), (uint32_t)kLRow);
                T Fn = T(1);
                if (mn < T(0)) Fn = cell_fraction(A, fy, C, fy - 2, tx, tp, row[kLTf]);
                const T dF = (fo - Fn) * rdt;
                fs = dF * row[kLCh];
                fl[k] = dF * row[kLCq];
                if (!(Fn == fo)) at<SMALL>(frac, idx) = Fn;
                if (!__builtin_isfinite(Fn)) st |= kStNonfinite;
            }
        }
        // (rows read by the reduction below)
        if (fy >= kHalo && fy < a.tile_y + kHalo) B[fy - 1][tx] = fs;
    }
    if (st) atomicOr(status, st);
    __syncthreads();

    // ---- step 6: mean flux over each atmosphere cell of the tile, summed
    // in a fixed order (columns, then the column sums)
    {
        const int fh = phase_copy(FH);
#pragma unroll
        for (int k = 0; k < KR; k++) {
            const int fy = ty + kNR * k;
            if (fy < fh) A[fy][tx] = fl[k];
        }
    }
    __syncthreads();
    const int nI = a.tile_x / a.sr_x, nJ = a.tile_y / a.sr_y;
    if (tx >= kHalo && tx < a.tile_x + kHalo) {
        for (int J = ty; J < nJ; J += kNR) {
            const int r0 = kHalo + J * a.sr_y;
            T s1 = T(0), s2 = T(0);
            for (int r = 0; r < a.sr_y; r++) {
                s1 += B[r0 + r - 1][tx];
                s2 += A[r0 + r][tx];
            }
            B[r0 - 1][tx] = s1;   // read above by this thread only
            A[r0][tx] = s2;
        }
    }
    __syncthreads();
    const int I0 = x0 / a.sr_x, J0 = y0 / a.sr_y;
    for (int q = tid; q < nI * nJ; q += kBlock) {
        const int J = q / nI, I = q - J * nI;
        const int IG = I0 + I, JG = J0 + J;
        if (IG >= a.nax || JG >= a.nay) continue;
        const int cx0 = x0 + I * a.sr_x, cy0 = y0 + J * a.sr_y;
        const int ncx = nx - cx0 < a.sr_x ? nx - cx0 : a.sr_x;
        const int ncy = ny - cy0 < a.sr_y ? ny - cy0 : a.sr_y;
        const int r0 = kHalo + J * a.sr_y, f0 = kHalo + I * a.sr_x;
        T s1 = T(0), s2 = T(0);
        for (int cI = 0; cI < a.sr_x; cI++) {
            s1 += B[r0 - 1][f0 + cI];
            s2 += A[r0][f0 + cI];
        }
        const T cnt = T(ncx * ncy);
        fsens[(size_t)JG * a.nax + IG] = s1 / cnt;
        flat[(size_t)JG * a.nax + IG] = s2 / cnt;
    }
}


// One fire domain: work-group b takes tile (b % 8) * per_xcd + b / 8, so each
// of the eight XCDs sweeps a contiguous band of row-major tiles and halo rows
// stay in its L2.
// Minimum waves per SIMD asked of the register allocator.  The ensemble
// kernel at the default FP32 120 x 20 tile (KR = 7: 39 KiB of frames plus
// its in-kernel ignition scratch) fits three work-groups of 8 waves per CU,
// i.e. 6 waves per SIMD, which needs <= 80 VGPRs; it lands a few registers
// above that unless asked.  Elsewhere the same request would force scratch
// spills, so nothing is asked (1).
template <typename T, int KR> constexpr int waves_per_simd() {
    return (sizeof(T) == 4 && KR == 7) ? 6 : 1;
}
// The plain step at that tile (no ignition scratch in LDS: its set-up comes
// from k_ign_plain) needs under 40 KiB, so four work-groups fit per CU, i.e.
// 8 waves per SIMD, within 64 VGPRs and the scalar registers of 8 waves.
template <typename T, int KR> constexpr int step_waves() {
    return (sizeof(T) == 4 && KR == 7) ? 8 : waves_per_simd<T, KR>();
}

// REC: the replay of a recorded run for its reverse pass.  Writes psi^{n+1},
// psi' (after ignition) and psi* (Heun stage 1) of every node and stops
// there: ignition times, fuel fraction and fluxes are not recomputed.
// mark (plain steps): where non-null, the step index a.mark_step is stored at
// every node whose ignition time this step sets.  The ignition set-up of
// the tiles comes from k_ign_plain (iuse, ilb, irow; read only while an
// ignition is active).
template <typename T, int KR, bool SMALL, bool REC>
__global__ void __launch_bounds__(kBlock, (step_waves<T, KR>()))
k_step(const StepArgs a, const IgnTable<T> *itab, const T *__restrict__ psi_in,
       T *__restrict__ psi_out, T *tign, T *frac, const T *__restrict__ uw,
       const T *__restrict__ vw, const T *__restrict__ dzdx, const T *__restrict__ dzdy,
       const uint8_t *__restrict__ cat, const T *__restrict__ coef, T *__restrict__ fsens,
       T *__restrict__ flat, int *status, T *__restrict__ rec_p0, T *__restrict__ rec_b,
       int32_t *__restrict__ mark, const uint32_t *__restrict__ iuse, const T *__restrict__ ilb,
       const T *__restrict__ irow) {
    const int bid = blockIdx.x;
    const int tile = (bid & 7) * a.per_xcd + (bid >> 3);
    if (tile >= a.ntiles) return;
    step_tile<T, KR, SMALL, REC, true>(a, tile, threadIdx.x, threadIdx.y, 0u, a.t, itab, psi_in,
                                       psi_out, tign, frac, uw, vw,
                                       dzdx, dzdy, cat, coef, fsens, flat, status, rec_p0, rec_b,
                                       mark, iuse, ilb, irow);
}

// An ensemble of domains in one launch: the tiles of all domains form one
// work list (domain-major), mapped onto the XCDs like a single domain; each
// work-group finds its domain, whose arrays sit at that domain's offsets in
// the concatenated buffers.  The model time is read from device memory so a
// step can be captured once and replayed.
// Work-list tile g of an ensemble launch: finds its member, whose arrays sit
// at that member's offsets in the concatenated buffers, and steps the tile.
// The model time is read from device memory so a step can be captured once
// and replayed.
template <typename T, int KR, bool SMALL>
__device__ __forceinline__ void
ens_tile(const StepArgs &common, const int g, const int tx, const int ty,
         const EnsDomain *__restrict__ doms,
         const int32_t *__restrict__ tile_dom, const EnsClock *__restrict__ clock,
         const char *__restrict__ itabs, T *psi_a, T *psi_b, T *tign, T *frac,
         const T *__restrict__ uw, const T *__restrict__ vw, const T *__restrict__ dzdx,
         const T *__restrict__ dzdy, const uint8_t *__restrict__ cat, const T *__restrict__ coef,
         T *__restrict__ fsens, T *__restrict__ flat, int *status) {
    // one member per work-group: keep its index (and so every field of its
    // table row) in scalar registers
    const int di = __builtin_amdgcn_readfirstlane(tile_dom[g]);
    const EnsDomain &d = doms[di];
    StepArgs a = common;
    a.nx = d.nx;
    a.ny = d.ny;
    a.tiles_x = d.tiles_x;
    a.nax = d.nax;
    a.nay = d.nay;
    // ignitions only inside the window of their activity (none outside)
    const double tw = clock->t;
    a.nign = (tw >= d.t_ign_lo && tw <= d.t_ign_hi) ? d.nign : 0;
    a.dx = d.dx;
    a.dy = d.dy;
    a.rdx = d.rdx;
    a.rdy = d.rdy;
    // the member's ignition geometry for this step (kIgnTableBytes apart)
    const IgnTable<T> *itab =
        reinterpret_cast<const IgnTable<T> *>(itabs + (size_t)di * kIgnTableBytes);
    const double tnow = clock->t;
    const bool flip = clock->cur != 0;
    const T *pin = flip ? psi_b : psi_a;
    T *pout = flip ? psi_a : psi_b;
    const size_t a0 = (size_t)d.atm_off;
    if (SMALL) {
        // the member's first element goes into the 32-bit element index, so
        // the array bases stay the launch's (no per-member 64-bit pointers)
        step_tile<T, KR, SMALL, false, false>(a, g - d.tile0, tx, ty, (uint32_t)d.cell_off,
                                              tnow, itab, pin,
                                              pout, tign, frac, uw, vw, dzdx, dzdy, cat, coef,
                                              fsens + a0, flat + a0, status + di, nullptr,
                                              nullptr, nullptr, nullptr, nullptr, nullptr);
    } else {
        const size_t c0 = (size_t)d.cell_off;
        step_tile<T, KR, SMALL, false, false>(a, g - d.tile0, tx, ty, 0u, tnow, itab, pin + c0,
                                              pout + c0,
                                              tign + c0, frac + c0, uw + c0, vw + c0, dzdx + c0,
                                              dzdy + c0, cat + c0, coef, fsens + a0, flat + a0,
                                              status + di, nullptr, nullptr, nullptr, nullptr,
                                              nullptr, nullptr);
    }
}

// An ensemble of domains in one launch, one work-group per tile: the tiles of
// all members form one work list (member-major), mapped onto the XCDs like a
// single domain.
template <typename T, int KR, bool SMALL>
__global__ void __launch_bounds__(kBlock, (waves_per_simd<T, KR>()))
k_ens_step(const StepArgs common, const EnsDomain *__restrict__ doms,
           const int32_t *__restrict__ tile_dom, const EnsClock *__restrict__ clock,
           const char *__restrict__ itabs, T *psi_a, T *psi_b, T *tign, T *frac,
           const T *__restrict__ uw, const T *__restrict__ vw, const T *__restrict__ dzdx,
           const T *__restrict__ dzdy, const uint8_t *__restrict__ cat,
           const T *__restrict__ coef, T *__restrict__ fsens, T *__restrict__ flat,
           int *status) {
    const int bid = blockIdx.x;
    const int g = (bid & 7) * common.per_xcd + (bid >> 3);
    if (g >= common.ntiles) return;
    ens_tile<T, KR, SMALL>(common, g, threadIdx.x, threadIdx.y, doms, tile_dom, clock, itabs,
                           psi_a, psi_b, tign, frac, uw, vw, dzdx, dzdy, cat, coef, fsens, flat,
                           status);
}

// The same step with resident work-groups: the grid is as many work-groups
// as fit on the device at once, and each takes tiles of its XCD's band of the
// work list (band = blockIdx % 8, as in k_ens_step) from a per-band counter
// until the band is done.  The counters are cleared by k_ign_geo, which runs
// before this kernel in stream order.  The next tile index is fetched while
// the current tile computes; every work-group leaves once its band's counter
// has passed the band's end, so the grid drains whatever its size.
// Waves per SIMD asked of the resident kernel: as for the one-shot kernels,
// and for the taller FP32 frames (KR >= 9, two work-groups per CU by LDS) the
// four waves that two work-groups need.
template <typename T, int KR> constexpr int persist_waves() {
    return (sizeof(T) == 4 && KR >= 9) ? 4 : waves_per_simd<T, KR>();
}

template <typename T, int KR, bool SMALL>
__global__ void __launch_bounds__(kBlock, (persist_waves<T, KR>()))
k_ens_persist(const StepArgs common, const EnsDomain *__restrict__ doms,
              const int32_t *__restrict__ tile_dom, const EnsClock *__restrict__ clock,
              const char *__restrict__ itabs, T *psi_a, T *psi_b, T *tign, T *frac,
              const T *__restrict__ uw, const T *__restrict__ vw, const T *__restrict__ dzdx,
              const T *__restrict__ dzdy, const uint8_t *__restrict__ cat,
              const T *__restrict__ coef, T *__restrict__ fsens, T *__restrict__ flat,
              int *status, int32_t *counters) {
    __shared__ int next_tile;
    const int band = blockIdx.x & 7;
    const int lo = band * common.per_xcd;
    const int hi = min(lo + common.per_xcd, common.ntiles);
    const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
    int mine = 0;
    if (lead) mine = lo + atomicAdd(&counters[band], 1);
    for (;;) {
        // the previous tile's last reads of next_tile came before its first
        // barrier, so the leader may overwrite it here
        if (lead) next_tile = mine;
        __syncthreads();
        const int g = next_tile;
        if (g >= hi) break;
        if (lead) mine = lo + atomicAdd(&counters[band], 1);
        // the thread's frame coordinates pass through an opaque copy each
        // tile, so values derived from them are formed inside the loop rather
        // than held in registers across it
        int tx = threadIdx.x, ty = threadIdx.y;
        asm volatile("" : "+v"(tx), "+v"(ty));
        ens_tile<T, KR, SMALL>(common, g, tx, ty, doms, tile_dom, clock, itabs, psi_a, psi_b,
                               tign, frac, uw, vw, dzdx, dzdy, cat, coef, fsens, flat, status);
    }
}

// The step's ignition geometry (IgnTable) of each domain, ahead of the step
// kernel: one thread per (domain, ignition slot).  A single domain passes its
// records and time; an ensemble its member table and device clock, each
// member's records FIRE_MAX_IGNITIONS apart.
template <typename T>
__global__ void k_ign_geo(const fire_ignition *__restrict__ ign, int nign, double t,
                          const EnsDomain *__restrict__ doms, const EnsClock *__restrict__ clock,
                          int ndom, char *__restrict__ tabs, int32_t *counters) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // work counters of a resident-work-group ensemble step start at zero
    if (counters && i < 8) counters[i] = 0;
    const int di = i / FIRE_MAX_IGNITIONS, g = i - di * FIRE_MAX_IGNITIONS;
    if (di >= ndom) return;
    const int n = doms ? doms[di].nign : nign;
    const double tt = doms ? clock->t : t;
    IgnGeo<T> geo = {};
    bool on = false;
    if (g < n) on = ign_setup<T>(ign[(size_t)di * FIRE_MAX_IGNITIONS + g], tt, geo);
    IgnTable<T> *tab = reinterpret_cast<IgnTable<T> *>(tabs + (size_t)di * kIgnTableBytes);
    tab->g[g] = geo;
    tab->on[g] = on ? 1 : 0;
}

// A single domain's ignition set-up for the step at time t (IgnSetLayout),
// ahead of the step kernel: every work-group forms the geometry of the
// ignitions (work-group 0 also writes the table the step reads), then thread
// i takes tile i (below the capacity) and table row i.  fhm: frame rows of
// the step kernel (its bounds cover the whole frame).
template <typename T>
__global__ void __launch_bounds__(256)
k_ign_plain(const fire_ignition *__restrict__ ign, int nign, double t, const StepArgs a,
            int fhm, IgnTable<T> *__restrict__ tab, uint32_t *__restrict__ iuse,
            T *__restrict__ ilb, T *__restrict__ irow) {
    __shared__ IgnGeo<T> geo[FIRE_MAX_IGNITIONS];
    __shared__ int on[FIRE_MAX_IGNITIONS];
    const int tid = threadIdx.x;
    if (tid < FIRE_MAX_IGNITIONS) {
        IgnGeo<T> gm = {};
        bool o = false;
        if (tid < nign) o = ign_setup<T>(ign[tid], t, gm);
        geo[tid] = gm;
        on[tid] = o ? 1 : 0;
        if (blockIdx.x == 0) {
            tab->g[tid] = gm;
            tab->on[tid] = o ? 1 : 0;
        }
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + tid;
    const int ncap = a.ntiles < a.tile_cap ? a.ntiles : a.tile_cap;
    if (i < ncap) {
        const int tyi = i / a.tiles_x, txi = i - tyi * a.tiles_x;
        const int fx0 = txi * a.tile_x - kHalo, fy0 = tyi * a.tile_y - kHalo;
        T lb[FIRE_MAX_IGNITIONS], ub[FIRE_MAX_IGNITIONS];
        for (int g = 0; g < nign; g++)
            if (on[g]) ign_frame_bounds(geo[g], fx0, fy0, fhm, a.dx, a.dy, lb[g], ub[g]);
        uint32_t word = 0;
        for (int g = 0; g < nign; g++) {
            if (!on[g]) continue;
            int use = 2;
            if (lb[g] > T(0)) {
                // psi_g > 0 on every frame node: it lights no node there; and
                // it is never the minimum where another active ignition's
                // psi_g is below it everywhere
                use = 1;
                for (int h = 0; h < nign; h++)
                    if (h != g && on[h] && ub[h] < lb[g]) use = 0;
            }
            word |= (uint32_t)use << (2 * g);
            ilb[(size_t)i * FIRE_MAX_IGNITIONS + g] = lb[g];
        }
        iuse[i] = word;
    }
    if (i == 0) {   // tiles past the capacity: every active ignition in full
        uint32_t word = 0;
        for (int g = 0; g < nign; g++)
            if (on[g]) word |= 2u << (2 * g);
        iuse[a.tile_cap] = word;
    }
    if (i < a.ign_rows) {
        for (int g = 0; g < nign; g++) {
            if (!on[g]) continue;
            const T py = ign_py(geo[g], i - kHalo, a.dy);
            irow[(size_t)g * a.ign_rows + i] = py;
            irow[(size_t)(FIRE_MAX_IGNITIONS + g) * a.ign_rows + i] = ign_by(geo[g], py);
        }
    }
}

// Advances an ensemble's device clock after its step kernel (stream order).
__global__ void k_advance_clock(EnsClock *c, double dt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->t += dt;
        c->cur ^= 1;
    }
}

// ---------------------------------------------------------------- init kernels

template <typename T>
__global__ void k_fill(T *psi, T *tign, T *frac, size_t n, T psi0) {
    const T INF = M<T>::inf();
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        psi[i] = psi0;
        tign[i] = INF;
        frac[i] = T(1);
    }
}

// Per-category coefficients of Eq. (3) from the fuel data (Table 1) via the
// Rothermel chain of Table 2 in English units, in double precision; plus
// T_f (Eq. 4) and the flux factors of Eqs. (5)-(6).  One thread per category.
template <typename T>
__global__ void k_coef(const fire_fuel *fuels, int ncat, double wind_cap, T *coef) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncat) return;
    const fire_fuel f = fuels[k];
    constexpr double ft = 0.3048, lb = 0.45359237, btu = 1055.05585262;
    constexpr double ftmin = ft / 60.0;  // m/s per ft/min
    constexpr double Lw = 2.5e6;         // J/kg, latent heat (Sect. 2.3)
    const double Mf = f.fuelmc_g;
    double out[kNCoef];
    out[kTf] = f.tf > 0.0 ? f.tf : f.weight * (-0.6 / ::log(0.6));
    out[kCh] = f.fgi * f.cmbcnst / (1.0 + Mf);
    out[kCq] = Lw * f.fgi * (Mf + 0.56) / (1.0 + Mf);
    out[kM] = f.ros_mult;
    if (f.ichap) {
        // Eq. (2): S = min{6, max{0.03333, 1.2974 U}} in coefficient form
        out[kS0] = 0.03333;
        out[kR0] = 0.0;
        out[kB] = 1.0;
        out[kC] = 1.2974;
        out[kD] = 0.0;
        out[kE] = 6.0 / 1.2974;
    } else {
        // English units (lb, ft, min, BTU)
        const double sig = f.savr * ft;
        const double load = f.fgi * (ft * ft / lb) / (1.0 + Mf);     // w_0
        const double rho_b = load / (f.fueldepthm / ft);
        const double beta = rho_b / (f.fueldens * (ft * ft * ft / lb));
        const double beta_op = 3.348 * ::pow(sig, -0.8189);
        const double ratio = beta / beta_op;
        const double Aexp = 1.0 / (4.77 * ::pow(sig, 0.1) - 7.27);
        const double sig15 = ::pow(sig, 1.5);
        const double gam = sig15 / (495.0 + 0.0594 * sig15) * ::pow(ratio, Aexp) *
                           ::exp(Aexp * (1.0 - ratio));
        double rm = Mf / f.fuelmce;
        rm = rm < 1.0 ? rm : 1.0;
        const double eta_m = 1.0 + rm * (-2.59 + rm * (5.11 - 3.52 * rm));
        const double eta_s = 0.174 * ::pow(f.se, -0.19);
        const double heat = f.cmbcnst * (lb / btu);
        const double IR = gam * (load / (1.0 + f.st)) * heat * eta_m * eta_s;
        const double xi = ::exp((0.792 + 0.681 * ::sqrt(sig)) * (beta + 0.1)) / (192.0 + 0.2595 * sig);
        const double qig = 250.0 + 1116.0 * Mf;
        const double R0 = IR * xi / (rho_b * ::exp(-138.0 / sig) * qig) * ftmin;   // m/s
        const double Cw = 7.47 * ::exp(-0.133 * ::pow(sig, 0.55));
        const double Bw = 0.02526 * ::pow(sig, 0.54);
        const double Ew = 0.715 * ::exp(-3.59e-4 * sig);
        out[kS0] = 0.0;
        out[kR0] = R0;
        out[kB] = Bw;
        out[kC] = R0 * Cw * ::pow(ratio, -Ew) * ::pow(f.windrf / ftmin, Bw);
        out[kD] = R0 * 5.275 * ::pow(beta, -0.3);
        out[kE] = wind_cap;
    }
    for (int j = 0; j < kNCoef; j++) coef[k * kNCoef + j] = T(out[j]);
}

template <typename T>
__global__ void k_ros_eval(const T *coef, int ncat, T cap, const uint8_t *cat, const T *un,
                           const T *tn, T *S, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int k = cat[i] < ncat ? cat[i] : 0;
        S[i] = ros(coef + k * kNCoef, un[i], tn[i], cap);
    }
}

template <typename T> __global__ void k_to_f64(const T *src, double *dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)src[i];
}

template <typename T, int KR, bool SMALL>
hipError_t launch_one(const StepArgs &a, const StepBuffers &b, hipStream_t s) {
    const size_t dyn = (size_t)a.ncat * kLRow * sizeof(T);
    const int grid = a.per_xcd * 8;
    // the ignition geometry of the step: every step of an ensemble (its time
    // is on the device), a single domain's only while an ignition is active
    const char *iset = (const char *)b.ign_set;
    const IgnSetLayout IL = ign_set_layout(a.tile_cap, a.ny, sizeof(T));
    const uint32_t *iuse = iset ? (const uint32_t *)(iset + IL.use) : nullptr;
    const T *ilb = iset ? (const T *)(iset + IL.lb) : nullptr;
    const T *irow = iset ? (const T *)(iset + IL.rows) : nullptr;
    if (!b.ens_doms && a.nign > 0) {
        if (!iset || a.tile_cap < 0 || a.ign_rows < a.ny + kFHMax) return hipErrorInvalidValue;
        const int nth = (a.ntiles < a.tile_cap ? a.ntiles : a.tile_cap) + 1;
        const int n = nth > a.ign_rows ? nth : a.ign_rows;
        hipLaunchKernelGGL((k_ign_plain<T>), dim3((n + 255) / 256), dim3(256), 0, s, b.ign,
                           a.nign, a.t, a, kNR * KR, (IgnTable<T> *)b.ign_tab,
                           (uint32_t *)iuse, (T *)ilb, (T *)irow);
    } else if (b.ens_doms) {
        const int nth = b.ndom * FIRE_MAX_IGNITIONS;
        hipLaunchKernelGGL((k_ign_geo<T>), dim3((nth + 63) / 64), dim3(64), 0, s, b.ign,
                           a.nign, a.t, b.ens_doms, b.ens_clock, b.ens_doms ? b.ndom : 1,
                           (char *)b.ign_tab, b.ens_slots > 0 ? b.ens_counters : nullptr);
    }
    if (b.ens_doms && b.ens_slots > 0) {
        hipLaunchKernelGGL((k_ens_persist<T, KR, SMALL>), dim3(b.ens_slots), dim3(kFW, kNR), dyn,
                           s, a, b.ens_doms, b.ens_tile_dom, b.ens_clock, (const char *)b.ign_tab,
                           (T *)b.psi_in, (T *)b.psi_out, (T *)b.tign, (T *)b.frac,
                           (const T *)b.u, (const T *)b.v, (const T *)b.dzdx, (const T *)b.dzdy,
                           b.cat, (const T *)b.coef, (T *)b.fsens, (T *)b.flat, b.status,
                           b.ens_counters);
    } else if (b.ens_doms) {
        hipLaunchKernelGGL((k_ens_step<T, KR, SMALL>), dim3(grid), dim3(kFW, kNR), dyn, s, a,
                           b.ens_doms, b.ens_tile_dom, b.ens_clock, (const char *)b.ign_tab,
                           (T *)b.psi_in,
                           (T *)b.psi_out, (T *)b.tign, (T *)b.frac, (const T *)b.u,
                           (const T *)b.v, (const T *)b.dzdx, (const T *)b.dzdy, b.cat,
                           (const T *)b.coef, (T *)b.fsens, (T *)b.flat, b.status);
    } else if (b.rec_p0) {
        hipLaunchKernelGGL((k_step<T, KR, SMALL, true>), dim3(grid), dim3(kFW, kNR), dyn, s, a,
                           (const IgnTable<T> *)b.ign_tab, (const T *)b.psi_in, (T *)b.psi_out,
                           (T *)b.tign, (T *)b.frac, (const T *)b.u, (const T *)b.v,
                           (const T *)b.dzdx, (const T *)b.dzdy, b.cat, (const T *)b.coef,
                           (T *)b.fsens, (T *)b.flat, b.status, (T *)b.rec_p0, (T *)b.rec_b,
                           (int32_t *)nullptr, iuse, ilb, irow);
    } else {
        hipLaunchKernelGGL((k_step<T, KR, SMALL, false>), dim3(grid), dim3(kFW, kNR), dyn, s, a,
                           (const IgnTable<T> *)b.ign_tab, (const T *)b.psi_in, (T *)b.psi_out,
                           (T *)b.tign, (T *)b.frac, (const T *)b.u, (const T *)b.v,
                           (const T *)b.dzdx, (const T *)b.dzdy, b.cat, (const T *)b.coef,
                           (T *)b.fsens, (T *)b.flat, b.status, (T *)nullptr, (T *)nullptr,
                           b.mark, iuse, ilb, irow);
    }
    return hipGetLastError();
}

template <typename T, int KR>
hipError_t step_k(const StepArgs &a, const StepBuffers &b, hipStream_t s) {
    // 32-bit byte offsets when every (concatenated) array is below 4 GiB
    const bool small = (uint64_t)b.ncells * sizeof(T) < ((uint64_t)1 << 32);
    return small ? launch_one<T, KR, true>(a, b, s) : launch_one<T, KR, false>(a, b, s);
}

// frame height tile_y + 6 <= 4 KR
template <typename T>
hipError_t step_t(const StepArgs &a, const StepBuffers &b, hipStream_t s) {
    const int fh = a.tile_y + 2 * kHalo;
    if (fh <= 16) return step_k<T, 4>(a, b, s);
    if (fh <= 20) return step_k<T, 5>(a, b, s);
    if (fh <= 24) return step_k<T, 6>(a, b, s);
    if (fh <= 28) return step_k<T, 7>(a, b, s);
    if (fh <= 32) return step_k<T, 8>(a, b, s);
    if constexpr (sizeof(T) == 4) {
        if (fh <= 36) return step_k<T, 9>(a, b, s);
        if (fh <= 40) return step_k<T, 10>(a, b, s);
        if (fh <= 44) return step_k<T, 11>(a, b, s);
        return step_k<T, 12>(a, b, s);
    }
    return hipErrorInvalidValue;
}

// Work-groups of k_ens_persist resident on the current device at once
// (occupancy times compute units, rounded down to a multiple of the eight
// XCD bands; 0 if the query fails).
template <typename T, int KR>
int persist_slots_k(int ncat, size_t ncells) {
    const size_t dyn = (size_t)ncat * kLRow * sizeof(T);
    const bool small = (uint64_t)ncells * sizeof(T) < ((uint64_t)1 << 32);
    int nb = 0, dev = 0, ncu = 0;
    const void *fn = small ? (const void *)k_ens_persist<T, KR, true>
                           : (const void *)k_ens_persist<T, KR, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, dyn) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return nb * ncu / 8 * 8;
}

template <typename T> int persist_slots_t(int tile_y, int ncat, size_t ncells) {
    const int fh = tile_y + 2 * kHalo;
    if (fh <= 16) return persist_slots_k<T, 4>(ncat, ncells);
    if (fh <= 20) return persist_slots_k<T, 5>(ncat, ncells);
    if (fh <= 24) return persist_slots_k<T, 6>(ncat, ncells);
    if (fh <= 28) return persist_slots_k<T, 7>(ncat, ncells);
    if (fh <= 32) return persist_slots_k<T, 8>(ncat, ncells);
    if constexpr (sizeof(T) == 4) {
        if (fh <= 36) return persist_slots_k<T, 9>(ncat, ncells);
        if (fh <= 40) return persist_slots_k<T, 10>(ncat, ncells);
        if (fh <= 44) return persist_slots_k<T, 11>(ncat, ncells);
        return persist_slots_k<T, 12>(ncat, ncells);
    }
    return 0;
}

}  // namespace

int persist_slots(int dtype, int tile_y, int ncat, size_t ncells) {
    return dtype == FIRE_F64 ? persist_slots_t<double>(tile_y, ncat, ncells)
                             : persist_slots_t<float>(tile_y, ncat, ncells);
}

hipError_t launch_step(int dtype, const StepArgs &a, const StepBuffers &b, hipStream_t s) {
    return dtype == FIRE_F64 ? step_t<double>(a, b, s) : step_t<float>(a, b, s);
}

hipError_t launch_advance_clock(EnsClock *c, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_advance_clock, dim3(1), dim3(64), 0, s, c, dt);
    return hipGetLastError();
}

hipError_t launch_coef(int dtype, const fire_fuel *fuels_dev, int ncat, double wind_cap,
                       void *coef_dev, hipStream_t s) {
    const int blk = 64, grid = (ncat + blk - 1) / blk;
    if (dtype == FIRE_F64)
        hipLaunchKernelGGL((k_coef<double>), dim3(grid), dim3(blk), 0, s, fuels_dev, ncat,
                           wind_cap, (double *)coef_dev);
    else
        hipLaunchKernelGGL((k_coef<float>), dim3(grid), dim3(blk), 0, s, fuels_dev, ncat,
                           wind_cap, (float *)coef_dev);
    return hipGetLastError();
}

hipError_t launch_fill(int dtype, void *psi, void *tign, void *frac, size_t n, double psi0,
                       hipStream_t s) {
    const int blk = 256;
    size_t g = (n + blk - 1) / blk;
    const int grid = (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
    if (dtype == FIRE_F64)
        hipLaunchKernelGGL((k_fill<double>), dim3(grid), dim3(blk), 0, s, (double *)psi,
                           (double *)tign, (double *)frac, n, psi0);
    else
        hipLaunchKernelGGL((k_fill<float>), dim3(grid), dim3(blk), 0, s, (float *)psi,
                           (float *)tign, (float *)frac, n, (float)psi0);
    return hipGetLastError();
}

hipError_t launch_ros_eval(int dtype, const void *coef, int ncat, double ros_cap,
                           const uint8_t *cat, const void *un, const void *tn, void *S,
                           int64_t n, hipStream_t s) {
    const int blk = 256;
    int64_t g = (n + blk - 1) / blk;
    const int grid = (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
    if (dtype == FIRE_F64)
        hipLaunchKernelGGL((k_ros_eval<double>), dim3(grid), dim3(blk), 0, s,
                           (const double *)coef, ncat, ros_cap, cat, (const double *)un,
                           (const double *)tn, (double *)S, n);
    else
        hipLaunchKernelGGL((k_ros_eval<float>), dim3(grid), dim3(blk), 0, s,
                           (const float *)coef, ncat, (float)ros_cap, cat, (const float *)un,
                           (const float *)tn, (float *)S, n);
    return hipGetLastError();
}

hipError_t launch_coef_to_f64(int dtype, const void *coef, double *out, int n, hipStream_t s) {
    const int blk = 256, grid = (n + blk - 1) / blk;
    if (dtype == FIRE_F64)
        hipLaunchKernelGGL((k_to_f64<double>), dim3(grid), dim3(blk), 0, s, (const double *)coef,
                           out, n);
    else
        hipLaunchKernelGGL((k_to_f64<float>), dim3(grid), dim3(blk), 0, s, (const float *)coef,
                           out, n);
    return hipGetLastError();
}

}  // namespace fire
