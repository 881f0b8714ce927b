// Reverse mode (adjoint) of the fire-mesh time step, and its C ABI.
//
// A differentiable run advances a context N steps with one surface wind
// (u, v) and step dt, keeping psi every K steps and, per node, the step in
// which its ignition time was set.  The backward pass takes dL/dF of the
// final fuel fraction and returns dL/du, dL/dv (per cell, summed over the
// steps), dL/dm_k (per-category spread multipliers) and dL/d(shift) of each
// ignition (translation of its segment or point).  Each segment of K steps
// is replayed with the forward kernel (bit-identical psi), then its steps are
// reversed one by one:
//
//   psi' = ignite(psi^n)                       (Sect. 4.4, min over ignitions)
//   psi* = psi' + dt F(G psi')                 (Eq. 11, stage 1)
//   psi^{n+1} = (psi' + psi*)/2 + dt/2 F(G psi*)   (stage 2)
//   t_i = t + psi' dt / (psi' - psi^{n+1})     (Eq. 14, nodes crossing in the step)
//   F_end = quadrature of Eqs. (15)-(19) on psi^N and t^
//
// with G the boundary extrapolation of Sect. 4.1 and F the right-hand side
// of Eqs. (12)-(13) with the spread rate of Eq. (3).  The discrete map is
// piecewise smooth; every branch (Godunov side, clamps and caps of the spread
// rate, ghost formula, ignition minimum, crossing step, sub-cell signs) is
// taken where the forward took it, and the derivative is that of the branch.
//
// The segment replay also records psi' and psi* of every step.  A reversed
// step is then three passes over the nodes: (1) the ignition times set in
// the step and the stage-2 partials, (2) their gather and the stage-1
// partials, (3) their gather and the ignition minimum.  A cell writes its
// five weighted stencil partials; every node gathers the ones aimed at it in
// a fixed order, plus its share of the side ghosts extrapolated from it (the
// transpose of G).  The final-time fuel fraction is reversed once, on
// ghost-extended arrays (its stencil reaches the corners).
// Gradients accumulate per cell in double and are reduced in a fixed order:
// results are bitwise reproducible and independent of K.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fire_device.h"

namespace fire {
namespace {

using namespace dev;

constexpr int kAB = 256;          // threads per block of the adjoint kernels
constexpr int kShift = 2 * FIRE_MAX_IGNITIONS;

struct AdjArgs {
    int32_t nx, ny, ncat, nign, visc_mode, ign_active;   // ign_active: some ignition at t
    double dx, dy, rdx, rdy, eps, cap, t, dt;
};

__device__ __forceinline__ int ext_idx(const AdjArgs &a, int x, int y) {
    return (y + 1) * (a.nx + 2) + (x + 1);
}

// The reverse step works on tiles of kRTX x kRTY nodes (one work-group of
// kAB threads, two nodes each).  Per-tile flags record where an array may be
// nonzero: dL/dpsi^{n+1} (two buffers, l1[0] / l1[1]), the crossing part of
// dL/dpsi' (lp0) and dL/dt_i (lt).  The adjoint of a run is nonzero only
// where the final fuel fraction depends on the state, a small part of the
// mesh; a tile whose inputs within reach are all zero has all-zero outputs,
// so it skips its work and only clears stale values.
constexpr int kRTX = 32, kRTY = 16;
constexpr int kREX = kRTX + 2, kREY = kRTY + 2;   // the tile and one ring
struct AdjFlags {
    int32_t *l1[2], *lp0, *lt;
};

__device__ __forceinline__ int rtiles_x(const AdjArgs &a) { return (a.nx + kRTX - 1) / kRTX; }
__device__ __forceinline__ int rtiles_y(const AdjArgs &a) { return (a.ny + kRTY - 1) / kRTY; }

// Whether tile t or one of its eight neighbours has its flag set (the
// reach of the ring's gathers, the ghost transposes included).
__device__ __forceinline__ bool nbhd_flag(const int32_t *f, const AdjArgs &a, int t) {
    const int tx = rtiles_x(a), ty = rtiles_y(a);
    const int cx = t % tx, cy = t / tx;
    bool any = false;
    for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
            const int x = cx + dx, y = cy + dy;
            if (x >= 0 && x < tx && y >= 0 && y < ty && f[y * tx + x]) any = true;
        }
    return any;
}

// d ghost(p, q) / d(p, q): ghost = 2p - q when p >= q, else q.
template <typename T> __device__ __forceinline__ void dghost(T p, T q, T &dp, T &dq) {
    if (p >= q) {
        dp = T(2);
        dq = T(-1);
    } else {
        dp = T(0);
        dq = T(1);
    }
}

// Right-hand side of Eq. (12) at a node and its derivatives with respect to
// the five stencil values, the wind components and the category multiplier.
// The forward value is computed exactly as rhs5 does.
template <typename T> struct RhsGrad {
    T F, dc, dw, de, ds, dn, du, dv, dm;
};

template <typename T>
__device__ RhsGrad<T> rhs5_grad(T pc, T pw, T pe, T ps, T pn, T u, T v, T gzx, T gzy,
                                const T *row, const T *g, const Consts<T> &c) {
    RhsGrad<T> r;
    const T dmx = (pc - pw) * c.rdx, dpx = (pe - pc) * c.rdx;
    const T dmy = (pc - ps) * c.rdy, dpy = (pn - pc) * c.rdy;
    const T ax = vmax(dmx, T(0)), bx = vmin(dpx, T(0));
    const T ay = vmax(dmy, T(0)), by = vmin(dpy, T(0));
    const bool selx = ax * ax >= bx * bx, sely = ay * ay >= by * by;
    const T gx2 = vmax(ax * ax, bx * bx), gy2 = vmax(ay * ay, by * by);
    const T up = M<T>::sqrt(gx2 + gy2);
    const T cx = (pe - pw) * c.rdx, cy = (pn - ps) * c.rdy;
    const T cn2 = cx * cx + cy * cy;
    const T inv = cn2 > T(0) ? M<T>::rsqrt(cn2) : T(0);
    const T nx = cx * inv, ny = cy * inv;
    const T un = u * nx + v * ny, tn = gzx * nx + gzy * ny;
    // spread rate (ros_row) and its pieces
    const T e = row[kLE], b = row[kLB];
    const T U = vmin(vmax(un, T(0)), e);
    const T gg = vmax(tn, T(0));
    const T Ub = M<T>::powp(U, b);
    const T s = row[kLR0] + row[kLC] * Ub + row[kLD] * (gg * gg);
    const T S1 = vmax(s, row[kLS0]);
    const T S = vmin(S1, c.cap);
    const T lap = (dpx - dmx) + (dpy - dmy);
    const T visc = c.visc_mode == 0 ? c.eps * S * lap : c.eps * lap;
    r.F = visc - S * up;

    // dS/d(un), dS/d(tn), dS/dm along the branch taken
    const bool live = S1 < c.cap;
    const bool in_s = s >= row[kLS0];
    const T dS_dun = (live && in_s && un > T(0) && un < e && U > T(0))
                         ? row[kLC] * b * M<T>::div(Ub, U) : T(0);
    const T dS_dtn = (live && in_s && tn > T(0)) ? T(2) * row[kLD] * gg : T(0);
    const T dS_dm = live ? (in_s ? g[kR0] + g[kC] * Ub + g[kD] * (gg * gg) : g[kS0]) : T(0);
    // through the unit normal n = (cx, cy)/|.|
    const T Snx = dS_dun * u + dS_dtn * gzx, Sny = dS_dun * v + dS_dtn * gzy;
    T dS_dcx = T(0), dS_dcy = T(0);
    if (cn2 > T(0)) {
        dS_dcx = inv * ny * (ny * Snx - nx * Sny);
        dS_dcy = inv * nx * (nx * Sny - ny * Snx);
    }
    // Godunov magnitude
    T Uxm = T(0), Uxp = T(0), Uym = T(0), Uyp = T(0);
    if (up > T(0)) {
        const T iu = M<T>::div(T(1), up);
        if (selx) Uxm = ax * iu; else Uxp = bx * iu;
        if (sely) Uym = ay * iu; else Uyp = by * iu;
    }
    const T dF_dS = (c.visc_mode == 0 ? c.eps * lap : T(0)) - up;
    const T kl = c.visc_mode == 0 ? c.eps * S : c.eps;
    // d/d(pc, pw, pe, ps, pn) of up, lap and S
    const T up_c = c.rdx * (Uxm - Uxp) + c.rdy * (Uym - Uyp);
    const T up_w = -c.rdx * Uxm, up_e = c.rdx * Uxp, up_s = -c.rdy * Uym, up_n = c.rdy * Uyp;
    const T lp_c = T(-2) * (c.rdx + c.rdy);
    r.dc = kl * lp_c - S * up_c;
    r.dw = dF_dS * (-c.rdx * dS_dcx) + kl * c.rdx - S * up_w;
    r.de = dF_dS * (c.rdx * dS_dcx) + kl * c.rdx - S * up_e;
    r.ds = dF_dS * (-c.rdy * dS_dcy) + kl * c.rdy - S * up_s;
    r.dn = dF_dS * (c.rdy * dS_dcy) + kl * c.rdy - S * up_n;
    r.du = dF_dS * dS_dun * nx;
    r.dv = dF_dS * dS_dun * ny;
    r.dm = dF_dS * dS_dm;
    return r;
}

// Fuel fraction of one cell (Eqs. 15-19, as cell_fraction computes it) and
// its derivatives with respect to the nine node values of psi (gp) and of
// t^ (gq), p[b][a] / q[b][a] with b the row (south to north), a the column.
template <typename T>
__device__ void cell_fraction_grad(const T p[3][3], const T q[3][3], T tp, T rTf, T gp[3][3],
                                   T gq[3][3]) {
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
        for (int a = 0; a < 3; a++) gp[b][a] = gq[b][a] = T(0);
    const T pc = p[1][1], qc = q[1][1];
#pragma unroll
    for (int sb = 0; sb < 2; sb++)
#pragma unroll
        for (int sa = 0; sa < 2; sa++) {
            const int ax = 2 * sa, by = 2 * sb;
            const T pk[4] = {pc, T(0.5) * (pc + p[1][ax]), T(0.5) * (pc + p[by][1]),
                             T(0.25) * (pc + p[1][ax] + p[by][1] + p[by][ax])};
            const T qk[4] = {qc, T(0.5) * (qc + q[1][ax]), T(0.5) * (qc + q[by][1]),
                             T(0.25) * (qc + q[1][ax] + q[by][1] + q[by][ax])};
            T sum = T(0), asum = T(0), tau = T(0);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                sum += pk[k];
                asum += vabs(pk[k]);
                tau += pk[k] >= T(0) ? T(0) : (tp - qk[k]);
            }
            if (!(asum > T(0))) continue;
            const T beta = T(0.5) * (T(1) - M<T>::div(sum, asum));
            const T x = T(0.25) * tau * rTf;
            const T E = M<T>::one_m_exp_neg(x);
            const T ex = T(1) - E;   // exp(-x)
            // F = 1 - 1/4 sum_q beta_q E_q
            T dpk[4], dqk[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const T sg = pk[k] >= T(0) ? T(1) : T(-1);
                const T dbeta = T(-0.5) * M<T>::div(asum - sum * sg, asum * asum);
                dpk[k] = T(-0.25) * dbeta * E;
                dqk[k] = pk[k] >= T(0) ? T(0) : T(0.0625) * beta * ex * rTf;
            }
            // back to the nodes through the bilinear weights
            gp[1][1] += dpk[0] + T(0.5) * (dpk[1] + dpk[2]) + T(0.25) * dpk[3];
            gq[1][1] += dqk[0] + T(0.5) * (dqk[1] + dqk[2]) + T(0.25) * dqk[3];
            gp[1][ax] += T(0.5) * dpk[1] + T(0.25) * dpk[3];
            gq[1][ax] += T(0.5) * dqk[1] + T(0.25) * dqk[3];
            gp[by][1] += T(0.5) * dpk[2] + T(0.25) * dpk[3];
            gq[by][1] += T(0.5) * dqk[2] + T(0.25) * dqk[3];
            gp[by][ax] += T(0.25) * dpk[3];
            gq[by][ax] += T(0.25) * dqk[3];
        }
}

// Fixed-order sum over a block of kAB threads (thread 0 gets the total).
__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = kAB / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Threads of the reversed-step kernel: one per node of the tile and its
// ring (kREX kREY = 612 of them), in ten waves.
constexpr int kRT = 640;

// Fixed-order sum over the kRT threads of a block (every thread gets it):
// threads 512.. fold onto 0..127, then a halving tree.
__device__ __forceinline__ double block_sum_rt(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    if (t < kRT - 512) sh[t] += sh[t + 512];
    __syncthreads();
    for (int s = 256; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// shift_reduce over the kRT threads of a reversed-step block.
__device__ __forceinline__ void shift_reduce_rt(int g, double cx, double cy, int nign,
                                                double *acc, double *sh, int b) {
    const int any = __syncthreads_or(g >= 0);
    if (!any) return;
    for (int k = 0; k < nign; k++) {
        const double sx = block_sum_rt(g == k ? cx : 0.0, sh);
        const double sy = block_sum_rt(g == k ? cy : 0.0, sh);
        if (threadIdx.x == 0) {
            acc[(size_t)b * kShift + 2 * k] += sx;
            acc[(size_t)b * kShift + 2 * k + 1] += sy;
        }
    }
}

// Adds per-ignition (x, y) contributions of tile b into acc[b][2g+c].
__device__ __forceinline__ void shift_reduce(int g, double cx, double cy, int nign, double *acc,
                                             double *sh, int b) {
    const int any = __syncthreads_or(g >= 0);
    if (!any) return;
    for (int k = 0; k < nign; k++) {
        const double sx = block_sum(g == k ? cx : 0.0, sh);
        const double sy = block_sum(g == k ? cy : 0.0, sh);
        if (threadIdx.x == 0) {
            acc[(size_t)b * kShift + 2 * k] += sx;
            acc[(size_t)b * kShift + 2 * k + 1] += sy;
        }
    }
}

// ---------------------------------------------------------------- kernels

// Extended copy with the ghost ring of Sect. 4.1 (corners: x extrapolation
// of the ghost row), as the step kernel fills it.
template <typename T>
__global__ void __launch_bounds__(kAB) k_ext(const AdjArgs a, const T *src, T *dst) {
    const int ex = a.nx + 2, ey = a.ny + 2;
    const int j = blockIdx.x * kAB + threadIdx.x;
    if (j >= ex * ey) return;
    const int x = j % ex - 1, y = j / ex - 1;
    const bool xin = x >= 0 && x < a.nx, yin = y >= 0 && y < a.ny;
    const int sx = x < 0 ? 1 : -1, sy = y < 0 ? 1 : -1;
    const int nx = a.nx;
    T r;
    if (xin && yin) {
        r = src[y * nx + x];
    } else if (yin) {
        r = ghost(src[y * nx + x + sx], src[y * nx + x + 2 * sx]);
    } else if (xin) {
        r = ghost(src[(y + sy) * nx + x], src[(y + 2 * sy) * nx + x]);
    } else {
        const T r1 = ghost(src[(y + sy) * nx + x + sx], src[(y + 2 * sy) * nx + x + sx]);
        const T r2 = ghost(src[(y + sy) * nx + x + 2 * sx], src[(y + 2 * sy) * nx + x + 2 * sx]);
        r = ghost(r1, r2);
    }
    dst[j] = r;
}

template <typename T> __device__ __forceinline__ Consts<T> consts(const AdjArgs &a) {
    Consts<T> c;
    c.rdx = T(a.rdx);
    c.rdy = T(a.rdy);
    c.eps = T(a.eps);
    c.cap = T(a.cap);
    c.visc_mode = a.visc_mode;
    return c;
}

// Corner ghosts (x extrapolation of the ghost row) hand their adjoint to the
// two ghost-row nodes they came from.  One thread, corners in a fixed order.
template <typename T> __global__ void k_adj_corners(const AdjArgs a, const T *E, T *LE) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int xs[2] = {-1, a.nx}, ys[2] = {-1, a.ny};
    for (int cy = 0; cy < 2; cy++)
        for (int cx = 0; cx < 2; cx++) {
            const int x = xs[cx], y = ys[cy];
            const int sx = x < 0 ? 1 : -1;
            const int c = ext_idx(a, x, y), r1 = ext_idx(a, x + sx, y), r2 = ext_idx(a, x + 2 * sx, y);
            T dp, dq;
            dghost(E[r1], E[r2], dp, dq);
            const T l = LE[c];
            LE[r1] += l * dp;
            LE[r2] += l * dq;
            LE[c] = T(0);
        }
}

// Transpose of the side ghosts: interior node j gets its own extended
// adjoint plus the share of each side ghost extrapolated from it;
// out = b1 + h b2 + b3 + that (null bases count as zero).
template <typename T>
__device__ __forceinline__ T ghostT_node(const AdjArgs &a, const T *src, const T *LE, const T *b1,
                                         const T *b2, T h, const T *b3, int i) {
    const int nx = a.nx, ny = a.ny;
    const int x = i % nx, y = i / nx;
    T s = LE[ext_idx(a, x, y)];
    T dp, dq;
    if (x <= 1) {   // left ghost of row y: ghost(src(0, y), src(1, y))
        dghost(src[y * nx], src[y * nx + 1], dp, dq);
        s += LE[ext_idx(a, -1, y)] * (x == 0 ? dp : dq);
    }
    if (x >= nx - 2) {   // right ghost: ghost(src(nx-1, y), src(nx-2, y))
        dghost(src[y * nx + nx - 1], src[y * nx + nx - 2], dp, dq);
        s += LE[ext_idx(a, nx, y)] * (x == nx - 1 ? dp : dq);
    }
    if (y <= 1) {   // bottom ghost of column x
        dghost(src[x], src[nx + x], dp, dq);
        s += LE[ext_idx(a, x, -1)] * (y == 0 ? dp : dq);
    }
    if (y >= ny - 2) {   // top ghost
        dghost(src[(ny - 1) * nx + x], src[(ny - 2) * nx + x], dp, dq);
        s += LE[ext_idx(a, x, ny)] * (y == ny - 1 ? dp : dq);
    }
    if (b1) s += b1[i];
    if (b2) s += h * b2[i];
    if (b3) s += b3[i];
    return s;
}

template <typename T>
__global__ void __launch_bounds__(kAB)
k_adj_ghostT(const AdjArgs a, const T *src, const T *LE, const T *b1, const T *b2, T h,
             const T *b3, T *out) {
    const int i = blockIdx.x * kAB + threadIdx.x;
    if (i >= a.nx * a.ny) return;
    out[i] = ghostT_node(a, src, LE, b1, b2, h, b3, i);
}



// ---- fused reverse step: node values with the side ghosts of Sect. 4.1
// formed inline (a five-point stencil of an interior cell never reaches a
// corner), and the gather of stage partials with the transpose of those
// ghosts, in the same order as the extended-array kernels above.

template <typename T>
__device__ __forceinline__ T node_g(const AdjArgs &a, const T *P, int x, int y) {
    const int nx = a.nx, ny = a.ny;
    if (x < 0) return ghost(P[y * nx], P[y * nx + 1]);
    if (x >= nx) return ghost(P[y * nx + nx - 1], P[y * nx + nx - 2]);
    if (y < 0) return ghost(P[x], P[nx + x]);
    if (y >= ny) return ghost(P[(ny - 1) * nx + x], P[(ny - 2) * nx + x]);
    return P[y * nx + x];
}

// Sum of the stage partials (planes c, w, e, s, n of D) aimed at interior
// node (x, y), plus its share of the side ghosts extrapolated from it.  A
// cell whose adjoint weight W is zero wrote no partials (they are zero), so
// they are read only where W != 0.
template <typename T>
__device__ __forceinline__ T gather_node(const AdjArgs &a, const T *D, const T *W, const T *P,
                                         int x, int y) {
    const int nx = a.nx, ny = a.ny;
    const size_t n = (size_t)nx * ny;
    const int i = y * nx + x;
    T s = T(0);
    if (W[i] != T(0)) s += D[i];
    if (x + 1 < nx && W[i + 1] != T(0)) s += D[n + i + 1];
    if (x - 1 >= 0 && W[i - 1] != T(0)) s += D[2 * n + i - 1];
    if (y + 1 < ny && W[i + nx] != T(0)) s += D[3 * n + i + nx];
    if (y - 1 >= 0 && W[i - nx] != T(0)) s += D[4 * n + i - nx];
    T dp, dq;
    if (x <= 1 && W[y * nx] != T(0)) {
        dghost(P[y * nx], P[y * nx + 1], dp, dq);
        s += D[n + y * nx] * (x == 0 ? dp : dq);
    }
    if (x >= nx - 2 && W[y * nx + nx - 1] != T(0)) {
        dghost(P[y * nx + nx - 1], P[y * nx + nx - 2], dp, dq);
        s += D[2 * n + y * nx + nx - 1] * (x == nx - 1 ? dp : dq);
    }
    if (y <= 1 && W[x] != T(0)) {
        dghost(P[x], P[nx + x], dp, dq);
        s += D[3 * n + x] * (y == 0 ? dp : dq);
    }
    if (y >= ny - 2 && W[(ny - 1) * nx + x] != T(0)) {
        dghost(P[(ny - 1) * nx + x], P[(ny - 2) * nx + x], dp, dq);
        s += D[4 * n + (ny - 1) * nx + x] * (y == ny - 1 ? dp : dq);
    }
    return s;
}

// Derivatives of stage F at cell i on level set P (side ghosts inline).
template <typename T>
__device__ __forceinline__ RhsGrad<T> stage_grad(const AdjArgs &a, const T *P, int x, int y,
                                                 const T *u, const T *v, const T *gzx,
                                                 const T *gzy, const uint8_t *cat,
                                                 const T *coef) {
    const int i = y * a.nx + x;
    const int cv = cat[i] < a.ncat - 1 ? cat[i] : a.ncat - 1;
    alignas(16) T row[kLRow];
    make_row(coef + cv * kNCoef, row, T(a.cap));
    return rhs5_grad(P[i], node_g(a, P, x - 1, y), node_g(a, P, x + 1, y), node_g(a, P, x, y - 1),
                     node_g(a, P, x, y + 1), u[i], v[i], gzx[i], gzy[i], row, coef + cv * kNCoef,
                     consts<T>(a));
}

// The five stencil partials of stage F at cell i weighted by q = w lam, into
// D.  Nothing is written where lam = 0 (the gathers skip such cells).
template <typename T>
__device__ __forceinline__ void stage_D(const RhsGrad<T> &r, int i, size_t n, T q, T *D) {
    D[i] = q * r.dc;
    D[n + i] = q * r.dw;
    D[2 * n + i] = q * r.de;
    D[3 * n + i] = q * r.ds;
    D[4 * n + i] = q * r.dn;
}

// Ignition state of node (x, y) at the start of a step: psi' = min over the
// active ignitions (the last one lowering it is `sel`), and the ignition
// whose arrival time a node lit in this step takes (`tsel`).
template <typename T>
__device__ __forceinline__ void ignite_node(const AdjArgs &a, const fire_ignition *ign, T psi,
                                            int x, int y, int &sel, int &tsel) {
    T p = psi;
    const T pold = p;
    T tig = M<T>::inf();
    sel = tsel = -1;
    for (int g = 0; g < a.nign; g++) {
        IgnGeo<T> geo;
        if (!ign_setup<T>(ign[g], a.t, geo)) continue;
        const T py = ign_py(geo, y, a.dy);
        const int ch = ign_apply(geo, ign_px(geo, x, a.dx), py, ign_by(geo, py), p, tig);
        if (ch & 2) tsel = g;
        if (ch & 1) sel = g;
    }
    if (!(pold > T(0) && p <= T(0))) tsel = -1;
}

// Reverse, part 1 at node i for step n: the ignition time set in the step
// (Eq. 14 for a crossing node, the arrival time for a node lit by an
// ignition) passes dL/dt_i on; then the stage-2 partials weighted by
// dt/2 dL/dpsi^{n+1}.  Returns dL/dpsi^{n+1} with the crossing part added.
template <typename T>
__device__ __forceinline__ T rev1_node(const AdjArgs &a, int n, int i, int x, int y, T lam,
                                       const int32_t *set_step, const T *psi_n, const T *P0,
                                       const T *B, const T *pn1, T *LT, T *LP0, const T *u,
                                       const T *v, const T *gzx, const T *gzy,
                                       const uint8_t *cat, const T *coef,
                                       const fire_ignition *ign, T *D, int &g, double &cx,
                                       double &cy) {
    T lp0 = T(0);
    if (set_step[i] == n) {
        const T lt = LT[i];
        LT[i] = T(0);
        const T p = P0[i], q = pn1[i];
        if (p > T(0)) {
            const T D2 = (p - q) * (p - q);
            const T dt = T(a.dt);
            const T iD2 = M<T>::div(T(1), D2);
            lam += lt * dt * p * iD2;
            lp0 = -lt * dt * q * iD2;
        } else if (lt != T(0)) {
            int sg, k;
            ignite_node(a, ign, psi_n[i], x, y, sg, k);
            IgnGeo<T> geo;
            if (k >= 0 && ign_setup<T>(ign[k], a.t, geo)) {
                const T px = ign_px(geo, x, a.dx);
                const T py = ign_py(geo, y, a.dy);
                const IgnNear<T> nq = ign_near(geo, px, py, ign_by(geo, py));
                const bool sfree = nq.s > T(0) && nq.s < T(1);
                const T d = M<T>::sqrt(nq.d2);
                const T arr = fmaT(d, geo.invS, fmaT(nq.s, geo.lenv, geo.tg));
                if (arr < geo.t) {
                    // translating the ignition by delta moves the node by -delta
                    T ax_ = T(0), ay_ = T(0);
                    if (d > T(0)) {
                        ax_ = -geo.invS * M<T>::div(nq.qx, d);
                        ay_ = -geo.invS * M<T>::div(nq.qy, d);
                    }
                    if (sfree) {
                        ax_ -= geo.lenv * geo.exL;
                        ay_ -= geo.lenv * geo.eyL;
                    }
                    g = k;
                    cx = (double)(lt * ax_);
                    cy = (double)(lt * ay_);
                }
            }
        }
    }
    LP0[i] = lp0;
    if (lam != T(0))
        stage_D(stage_grad(a, B, x, y, u, v, gzx, gzy, cat, coef), i, (size_t)a.nx * a.ny,
                T(0.5) * T(a.dt) * lam, D);
    return lam;
}

// Sum of the stage-1 partials aimed at owned node (x, y), from the tile's
// LDS copy of dL/dpsi* (W) and of the partial planes (Dc, Dw, De, Ds, Dn) on
// the tile and its ring, plus its share of the side ghosts extrapolated from
// it: gather_node in the same order of terms.  (ex, ey) is the node's
// position in the ringed tile; P (psi') comes from memory for the ghost
// formula.
template <typename T>
__device__ __forceinline__ T gather_lds(const AdjArgs &a, const T (*W)[kREX],
                                        const T (*Dp)[kREY][kREX], const T *P, int x, int y,
                                        int ex, int ey, int x0, int y0) {
    const int nx = a.nx, ny = a.ny;
    T s = T(0);
    if (W[ey][ex] != T(0)) s += Dp[0][ey][ex];
    if (x + 1 < nx && W[ey][ex + 1] != T(0)) s += Dp[1][ey][ex + 1];
    if (x - 1 >= 0 && W[ey][ex - 1] != T(0)) s += Dp[2][ey][ex - 1];
    if (y + 1 < ny && W[ey + 1][ex] != T(0)) s += Dp[3][ey + 1][ex];
    if (y - 1 >= 0 && W[ey - 1][ex] != T(0)) s += Dp[4][ey - 1][ex];
    // the ghost sources sit in the ring: columns 0 / nx - 1, rows 0 / ny - 1
    const int gx0 = 0 - x0 + 1, gx1 = nx - 1 - x0 + 1;
    const int gy0 = 0 - y0 + 1, gy1 = ny - 1 - y0 + 1;
    T dp, dq;
    if (x <= 1 && W[ey][gx0] != T(0)) {
        dghost(P[y * nx], P[y * nx + 1], dp, dq);
        s += Dp[1][ey][gx0] * (x == 0 ? dp : dq);
    }
    if (x >= nx - 2 && W[ey][gx1] != T(0)) {
        dghost(P[y * nx + nx - 1], P[y * nx + nx - 2], dp, dq);
        s += Dp[2][ey][gx1] * (x == nx - 1 ? dp : dq);
    }
    if (y <= 1 && W[gy0][ex] != T(0)) {
        dghost(P[x], P[nx + x], dp, dq);
        s += Dp[3][gy0][ex] * (y == 0 ? dp : dq);
    }
    if (y >= ny - 2 && W[gy1][ex] != T(0)) {
        dghost(P[(ny - 1) * nx + x], P[(ny - 2) * nx + x], dp, dq);
        s += Dp[4][gy1][ex] * (y == ny - 1 ? dp : dq);
    }
    return s;
}

// Reverse, part 3 at owned node i for step n, given the gathered stage-1
// partials (gath) and dL/dpsi* (lb): dL/dpsi' = gathered partials + crossing part +
// dL/dpsi^{n+1}/2 + dL/dpsi*, then through the ignition minimum: returns
// dL/dpsi^n (zero where an ignition set psi', whose shift gets the
// contribution instead).
template <typename T>
__device__ __forceinline__ T rev3_lds(const AdjArgs &a, int i, int x, int y, T l1, T lb, T gath,
                                      const T *LP0, const T *psi_n, const fire_ignition *ign,
                                      int &g, double &cx, double &cy) {
    T l = gath;
    l += LP0[i];
    l += T(0.5) * l1;
    l += lb;
    int sg = -1, tg;
    if (a.ign_active) ignite_node(a, ign, psi_n[i], x, y, sg, tg);
    if (sg < 0) return l;
    IgnGeo<T> geo;
    if (l != T(0) && ign_setup<T>(ign[sg], a.t, geo)) {
        const T px = ign_px(geo, x, a.dx);
        const T py = ign_py(geo, y, a.dy);
        const IgnNear<T> nq = ign_near(geo, px, py, ign_by(geo, py));
        const T d = M<T>::sqrt(nq.d2);
        if (d > T(0)) {
            g = sg;
            cx = (double)(-l * M<T>::div(nq.qx, d));
            cy = (double)(-l * M<T>::div(nq.qy, d));
        }
    }
    return T(0);
}

// Part 1 alone of step n (the last step of a segment), tile by tile:
// dL/dpsi^{n+1} in L1 gets the crossing part of the nodes set in the step,
// the stage-2 partials go to D, LP0 and LT are updated.
template <typename T>
__global__ void __launch_bounds__(kAB)
k_rev_part1(const AdjArgs a, int n, const int32_t *set_step, const T *psi_n, const T *P0,
            const T *B, const T *pn1, T *L1, int32_t *f_l1, T *LT, T *LP0, const T *u,
            const T *v, const T *gzx, const T *gzy, const uint8_t *cat, const T *coef,
            const fire_ignition *ign, T *D, double *acc, AdjFlags fl) {
    __shared__ double sh[kAB];
    const int t = blockIdx.x;
    const int x0 = (t % rtiles_x(a)) * kRTX, y0 = (t / rtiles_x(a)) * kRTY;
    if (!f_l1[t] && !fl.lt[t]) {
        // lam and dL/dt_i zero on the tile: so is every output but stale LP0
        if (fl.lp0[t]) {
            for (int j = 0; j < 2; j++) {
                const int q = threadIdx.x + j * kAB;
                const int x = x0 + q % kRTX, y = y0 + q / kRTX;
                if (x < a.nx && y < a.ny) LP0[y * a.nx + x] = T(0);
            }
            if (threadIdx.x == 0) fl.lp0[t] = 0;
        }
        return;
    }
    bool n1 = false, np = false, nt = false;
    for (int j = 0; j < 2; j++) {
        const int q = threadIdx.x + j * kAB;
        const int x = x0 + q % kRTX, y = y0 + q / kRTX;
        int g = -1;
        double cx = 0.0, cy = 0.0;
        if (x < a.nx && y < a.ny) {
            const int i = y * a.nx + x;
            T l1 = L1[i];
            const T lam = rev1_node(a, n, i, x, y, l1, set_step, psi_n, P0, B, pn1, LT, LP0, u,
                                    v, gzx, gzy, cat, coef, ign, D, g, cx, cy);
            if (set_step[i] == n) {
                L1[i] = lam;
                l1 = lam;
            }
            n1 |= l1 != T(0);
            np |= LP0[i] != T(0);
            nt |= LT[i] != T(0);
        }
        shift_reduce(g, cx, cy, a.nign, acc, sh, t);
    }
    const int f1 = __syncthreads_or(n1);
    const int fp = __syncthreads_or(np);
    const int ft = __syncthreads_or(nt);
    if (threadIdx.x == 0) {
        f_l1[t] = f1;
        fl.lp0[t] = fp;
        fl.lt[t] = ft;
    }
}

// One reversed step n, tile by tile: part 2 (dL/dpsi* = dL/dpsi^{n+1}/2 +
// the stage-2 partials gathered through the ghosts of psi*, then the stage-1
// partials weighted by dt dL/dpsi*, with the wind and multiplier partials of
// both stages) on the tile and its ring into LDS, then part 3 (the gather of
// the stage-1 partials and the ignition minimum) on the tile, and, with
// part1, part 1 of step n - 1 at the same nodes.  Reads dL/dpsi^{n+1} from
// L1i and the stage-2 partials from Di; writes dL/dpsi^n (part 1 of step
// n - 1 applied) to L1o and that step's stage-2 partials to Do: the ring
// reads its neighbours' inputs, so those two are double-buffered.
template <typename T>
__global__ void __launch_bounds__(kRT)
k_rev_tile(const AdjArgs a2, const AdjArgs a1, int part1, int n1, const T *Di, const T *L1i,
           const int32_t *f_l1i, const T *B, const T *P0, const T *psi_n, T *LP0, T *L1o,
           int32_t *f_l1o, T *Do, const int32_t *set_step, const T *psi_n1, const T *P0n1,
           const T *Bn1, T *LT, const T *u, const T *v, const T *gzx, const T *gzy,
           const uint8_t *cat, const T *coef, const fire_ignition *ign, double *gu, double *gv,
           double *gm, double *acc, AdjFlags fl) {
    __shared__ T W[kREY][kREX];          // dL/dpsi* on the tile and its ring
    __shared__ T Dp[5][kREY][kREX];      // its stage-1 partials (c, w, e, s, n)
    __shared__ double sh[kRT];
    const AdjArgs &a = a2;
    const int nx = a.nx, ny = a.ny;
    const int t = blockIdx.x;
    const int x0 = (t % rtiles_x(a)) * kRTX, y0 = (t / rtiles_x(a)) * kRTY;
    const bool live = nbhd_flag(f_l1i, a, t) || fl.lp0[t] || (part1 && fl.lt[t]);
    if (!live) {
        // every output is zero: clear what the output buffer holds from two
        // steps ago
        if (f_l1o[t]) {
            const int q = threadIdx.x;
            const int x = x0 + q % kRTX, y = y0 + q / kRTX;
            if (q < kRTX * kRTY && x < nx && y < ny) L1o[y * nx + x] = T(0);
            if (threadIdx.x == 0) f_l1o[t] = 0;
        }
        return;
    }
    // ---- part 2 on the tile and its ring, one node per thread
    const int e = threadIdx.x;
    const int ex2 = e % kREX, ey2 = e / kREX;
    const int x2 = x0 - 1 + ex2, y2 = y0 - 1 + ey2;
    if (e < kREX * kREY && x2 >= 0 && x2 < nx && y2 >= 0 && y2 < ny) {
        const int ex = ex2, ey = ey2, x = x2, y = y2;
        const int i = y * nx + x;
        const T l1 = L1i[i];
        T lb = gather_node(a, Di, L1i, B, x, y);
        lb += T(0.5) * l1;
        W[ey][ex] = lb;
        const bool own = ex >= 1 && ex <= kRTX && ey >= 1 && ey <= kRTY;
        double du = 0.0, dv = 0.0, dm = 0.0;
        if (l1 != T(0) || lb != T(0)) {
            if (own) {
                du = gu[i];
                dv = gv[i];
                dm = gm[i];
            }
            if (own && l1 != T(0)) {
                // wind and multiplier partials of stage 2 (weight dt/2 lam^{n+1})
                const RhsGrad<T> r2 = stage_grad(a, B, x, y, u, v, gzx, gzy, cat, coef);
                const T q2 = T(0.5) * T(a.dt) * l1;
                du += (double)(q2 * r2.du);
                dv += (double)(q2 * r2.dv);
                dm += (double)(q2 * r2.dm);
            }
            if (lb != T(0)) {
                const RhsGrad<T> r1 = stage_grad(a, P0, x, y, u, v, gzx, gzy, cat, coef);
                const T q1 = T(a.dt) * lb;
                Dp[0][ey][ex] = q1 * r1.dc;
                Dp[1][ey][ex] = q1 * r1.dw;
                Dp[2][ey][ex] = q1 * r1.de;
                Dp[3][ey][ex] = q1 * r1.ds;
                Dp[4][ey][ex] = q1 * r1.dn;
                if (own) {
                    du += (double)(q1 * r1.du);
                    dv += (double)(q1 * r1.dv);
                    dm += (double)(q1 * r1.dm);
                }
            }
            if (own) {
                gu[i] = du;
                gv[i] = dv;
                gm[i] = dm;
            }
        }
    }
    __syncthreads();
    // ---- part 3 of step n, then part 1 of step n - 1, one tile node per thread
    bool nz1 = false, nzp = false, nzt = false;
    {
        const int q = threadIdx.x;
        const int ex = q % kRTX + 1, ey = q / kRTX + 1;
        const int x = x0 + ex - 1, y = y0 + ey - 1;
        int g3 = -1, g1 = -1;
        double cx3 = 0.0, cy3 = 0.0, cx1 = 0.0, cy1 = 0.0;
        if (q < kRTX * kRTY && x < nx && y < ny) {
            const int i = y * nx + x;
            const T gath = gather_lds(a, W, Dp, P0, x, y, ex, ey, x0, y0);
            const T l = rev3_lds(a, i, x, y, L1i[i], W[ey][ex], gath, LP0, psi_n, ign, g3, cx3,
                                 cy3);
            T lo = l;
            if (part1)
                lo = rev1_node(a1, n1, i, x, y, l, set_step, psi_n1, P0n1, Bn1, psi_n, LT, LP0,
                               u, v, gzx, gzy, cat, coef, ign, Do, g1, cx1, cy1);
            L1o[i] = lo;
            nz1 |= lo != T(0);
            nzp |= LP0[i] != T(0);
            nzt |= LT[i] != T(0);
        }
        shift_reduce_rt(g3, cx3, cy3, a.nign, acc, sh, t);
        shift_reduce_rt(g1, cx1, cy1, a1.nign, acc, sh, t);
    }
    const int f1 = __syncthreads_or(nz1);
    const int fp = __syncthreads_or(nzp);
    const int ft = __syncthreads_or(nzt);
    if (threadIdx.x == 0) {
        f_l1o[t] = f1;
        fl.lp0[t] = fp;
        fl.lt[t] = ft;
    }
}

// Per-tile flag of an array: whether any of the tile's values is nonzero.
template <typename T>
__global__ void __launch_bounds__(kAB) k_tile_any(const AdjArgs a, const T *p, int32_t *f) {
    const int t = blockIdx.x;
    const int x0 = (t % rtiles_x(a)) * kRTX, y0 = (t / rtiles_x(a)) * kRTY;
    bool any = false;
    for (int j = 0; j < 2; j++) {
        const int q = threadIdx.x + j * kAB;
        const int x = x0 + q % kRTX, y = y0 + q / kRTX;
        if (x < a.nx && y < a.ny) any |= p[y * a.nx + x] != T(0);
    }
    const int r = __syncthreads_or(any);
    if (threadIdx.x == 0) f[t] = r;
}

// Node times t^ on the extended mesh: t' where psi >= 0 and on the ghosts,
// else t_i (as the step kernel forms them for the fuel fraction).
template <typename T>
__global__ void __launch_bounds__(kAB)
k_that(const AdjArgs a, const T *psi, const T *tign, T tp, T *TH) {
    const int ex = a.nx + 2, ey = a.ny + 2;
    const int j = blockIdx.x * kAB + threadIdx.x;
    if (j >= ex * ey) return;
    const int x = j % ex - 1, y = j / ex - 1;
    T r = tp;
    if (x >= 0 && x < a.nx && y >= 0 && y < a.ny) {
        const int i = y * a.nx + x;
        r = psi[i] >= T(0) ? tp : tign[i];
    }
    TH[j] = r;
}

// dL/dpsi and dL/dt^ at extended node j from dL/dF of the (up to nine)
// interior cells whose fuel-fraction stencil holds it.
template <typename T>
__global__ void __launch_bounds__(kAB)
k_adj_frac(const AdjArgs a, const T *E, const T *TH, const T *lamF, const uint8_t *cat,
           const T *coef, T tp, T *LE, T *LTH) {
    const int ex = a.nx + 2, ey = a.ny + 2;
    const int j = blockIdx.x * kAB + threadIdx.x;
    if (j >= ex * ey) return;
    const int x = j % ex - 1, y = j / ex - 1;
    T sp = T(0), sq = T(0);
    for (int oy = -1; oy <= 1; oy++)
        for (int ox = -1; ox <= 1; ox++) {
            const int cx = x + ox, cy = y + oy;
            if (cx < 0 || cx >= a.nx || cy < 0 || cy >= a.ny) continue;
            const int ci = cy * a.nx + cx;
            const T lf = lamF[ci];
            if (lf == T(0)) continue;
            T p[3][3], q[3][3];
            T mn = M<T>::inf();
            for (int b = 0; b < 3; b++)
                for (int aa = 0; aa < 3; aa++) {
                    const int e = ext_idx(a, cx + aa - 1, cy + b - 1);
                    p[b][aa] = E[e];
                    q[b][aa] = TH[e];
                    mn = vmin(mn, p[b][aa]);
                }
            if (!(mn < T(0))) continue;   // F = 1 exactly there
            const int cv = cat[ci] < a.ncat - 1 ? cat[ci] : a.ncat - 1;
            const T rTf = T(1) / coef[cv * kNCoef + kTf];
            T gp[3][3], gq[3][3];
            cell_fraction_grad(p, q, tp, rTf, gp, gq);
            const int b = -oy + 1, aa = -ox + 1;   // node j within the cell's stencil
            sp += lf * gp[b][aa];
            sq += lf * gq[b][aa];
        }
    LE[j] = sp;
    LTH[j] = sq;
}

// dL/dt_i from dL/dt^ where t^ = t_i (psi < 0).
template <typename T>
__global__ void __launch_bounds__(kAB)
k_lt_init(const AdjArgs a, const T *psi, const T *LTH, T *LT) {
    const int i = blockIdx.x * kAB + threadIdx.x;
    if (i >= a.nx * a.ny) return;
    const int x = i % a.nx, y = i / a.nx;
    LT[i] = psi[i] < T(0) ? LTH[ext_idx(a, x, y)] : T(0);
}

template <typename T> __global__ void __launch_bounds__(kAB) k_set(T *p, T v, size_t cnt) {
    for (size_t i = blockIdx.x * (size_t)kAB + threadIdx.x; i < cnt; i += (size_t)gridDim.x * kAB)
        p[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(kAB) k_cast(const double *src, T *dst, int cnt) {
    const int i = blockIdx.x * kAB + threadIdx.x;
    if (i < cnt) dst[i] = T(src[i]);
}

// Per-block, per-category sums of gm (fixed order), then column sums.
__global__ void __launch_bounds__(kAB)
k_cat_partial(const double *gm, const uint8_t *cat, int cnt, int ncat, double *part) {
    __shared__ double sh[kAB];
    const int i = blockIdx.x * kAB + threadIdx.x;
    const double v = i < cnt ? gm[i] : 0.0;
    const int c = i < cnt ? (cat[i] < ncat - 1 ? cat[i] : ncat - 1) : -1;
    for (int k = 0; k < ncat; k++) {
        const int any = __syncthreads_or(c == k);
        if (!any) {
            if (threadIdx.x == 0) part[(size_t)blockIdx.x * ncat + k] = 0.0;
            continue;
        }
        const double s = block_sum(c == k ? v : 0.0, sh);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * ncat + k] = s;
    }
}

// out[k] = sum over rows of part[row][k]: one block per column, fixed order.
__global__ void __launch_bounds__(kAB)
k_col_sum(const double *part, int rows, int cols, double *out) {
    __shared__ double sh[kAB];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += kAB) s += part[(size_t)r * cols + k];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[k] = s;
}

// ---------------------------------------------------------------- host side

int hip_fail(hipError_t e) { return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP; }

struct AdjLayout {
    size_t ckpt, stack, rp0, rb, set_step, flux, e1, e2, le, th, l1, lt, lp0,
        lb, d, d1, gu, gv, gm, acc, part, small, flags, total;
};

}  // namespace
}  // namespace fire

using namespace fire;

struct fire_adj {
    fire_ctx *c;
    int nsteps, every, nseg;
    char *arena;
    AdjLayout L;
    std::vector<double> tstep;   // model time before step n (n = 0..nsteps)
    const void *u, *v;
    double dt;
    int forward_done;
    int nblk, nblk_ext;
    // The backward replays segment s - 1 on its own stream while segment s
    // is reversed on the context's stream, into the other of two sets of
    // replay buffers; events order the two.
    hipStream_t rs;
    hipEvent_t ev0, ev_rep[2], ev_rev[2];
};

namespace {

AdjLayout adj_layout(const fire_mesh *m, int ncat, int nsteps, int every) {
    const size_t n = (size_t)m->nx * m->ny, ne = (size_t)(m->nx + 2) * (m->ny + 2);
    const size_t es = esize(m);
    const size_t natm = (size_t)((m->nx + m->sr_x - 1) / m->sr_x) * ((m->ny + m->sr_y - 1) / m->sr_y);
    const int nseg = (nsteps + every - 1) / every;
    const size_t nblk = (n + kAB - 1) / kAB;
    AdjLayout L;
    size_t o = 0;
    auto take = [&](size_t &f, size_t bytes) {
        f = o;
        o = align_up(o + bytes);
    };
    take(L.ckpt, (size_t)nseg * n * es);
    take(L.stack, 2 * (size_t)(every + 1) * n * es);   // two sets: segment parity
    take(L.rp0, 2 * (size_t)every * n * es);
    take(L.rb, 2 * (size_t)every * n * es);
    take(L.set_step, n * 4);
    take(L.flux, 2 * natm * es);
    take(L.e1, ne * es);
    take(L.e2, ne * es);
    take(L.le, ne * es);
    take(L.th, ne * es);
    take(L.l1, n * es);
    take(L.lt, n * es);
    take(L.lp0, n * es);
    take(L.lb, n * es);
    take(L.d, 5 * n * es);
    take(L.d1, 5 * n * es);
    take(L.gu, n * 8);
    take(L.gv, n * 8);
    take(L.gm, n * 8);
    const size_t ntile = (size_t)((m->nx + kRTX - 1) / kRTX) * ((m->ny + kRTY - 1) / kRTY);
    take(L.acc, ntile * kShift * 8);
    take(L.part, nblk * (size_t)(ncat > kShift ? ncat : kShift) * 8);
    take(L.small, (size_t)(256 + kShift) * 8);
    take(L.flags, 4 * ntile * sizeof(int32_t));   // AdjFlags: l1[2], lp0, lt
    L.total = o;
    return L;
}

template <typename T> struct Run {
    fire_adj *A;
    fire_ctx *c;
    AdjArgs a;
    hipStream_t s;
    size_t n, ne;
    int gn, ge;

    template <typename P> P *at(size_t off) { return reinterpret_cast<P *>(A->arena + off); }
    T *arr(size_t off) { return at<T>(off); }
    // replay buffers of segment parity p: psi before step k of the segment,
    // psi' and psi* of step k
    T *stack(int p, int k) {
        return arr(A->L.stack) + ((size_t)p * (A->every + 1) + k) * n;
    }
    T *rp0(int p, int k) { return arr(A->L.rp0) + ((size_t)p * A->every + k) * n; }
    T *rb(int p, int k) { return arr(A->L.rb) + ((size_t)p * A->every + k) * n; }
    const T *coef() { return reinterpret_cast<const T *>(c->arena + c->off_coef); }
    const fire_ignition *ign() {
        return reinterpret_cast<const fire_ignition *>(c->arena + c->off_ign);
    }
    const T *cur_psi() { return reinterpret_cast<const T *>(c->arena + c->off_psi[c->cur]); }
    const T *tign_final() { return reinterpret_cast<const T *>(c->arena + c->off_tign); }
    // reverse-pass tiles, the per-tile flags, and the two buffers of
    // dL/dpsi^{n+1} and of the stage-2 partials (cur: the current one)
    int ntile() const {
        return ((c->mesh.nx + kRTX - 1) / kRTX) * ((c->mesh.ny + kRTY - 1) / kRTY);
    }
    AdjFlags flags() {
        int32_t *f = at<int32_t>(A->L.flags);
        const int nt = ntile();
        AdjFlags r;
        r.l1[0] = f;
        r.l1[1] = f + nt;
        r.lp0 = f + 2 * nt;
        r.lt = f + 3 * nt;
        return r;
    }
    int cur = 0;
    T *l1buf(int k) { return arr(k ? A->L.lb : A->L.l1); }
    T *dbuf(int k) { return arr(k ? A->L.d1 : A->L.d); }
    // whether any ignition is active at time t (the test of ign_setup)
    int ign_active_at(double t) const {
        for (int g = 0; g < c->nign; g++) {
            const fire_ignition &q = c->ign[g];
            const bool torch = q.vx != 0.0 || q.vy != 0.0;
            const double tend = torch ? q.t_end : q.t_start;
            const double grow = std::isinf(q.ros) ? 0.0 : q.radius / q.ros;
            if (t >= q.t_start && t <= tend + grow) return 1;
        }
        return 0;
    }

    explicit Run(fire_adj *A_) : A(A_), c(A_->c), s(A_->c->stream) {
        const fire_mesh &m = c->mesh;
        std::memset(&a, 0, sizeof(a));
        a.nx = m.nx;
        a.ny = m.ny;
        a.ncat = c->ncat;
        a.nign = c->nign;
        a.visc_mode = c->prm.viscosity_mode;
        a.dx = m.dx;
        a.dy = m.dy;
        a.rdx = 1.0 / m.dx;
        a.rdy = 1.0 / m.dy;
        a.eps = c->prm.viscosity;
        a.cap = c->prm.ros_cap;
        a.dt = A->dt;
        n = (size_t)m.nx * m.ny;
        ne = (size_t)(m.nx + 2) * (m.ny + 2);
        gn = (int)((n + kAB - 1) / kAB);
        ge = (int)((ne + kAB - 1) / kAB);
    }

    hipError_t zero_d(size_t off, size_t cnt) {
        hipLaunchKernelGGL(k_set<double>, dim3(256), dim3(kAB), 0, s, at<double>(off), 0.0, cnt);
        return hipGetLastError();
    }

    // dL/dpsi^N and dL/dt_i from dL/dF_end
    hipError_t loss_init(const T *dF) {
        const T *psiN = cur_psi();
        const T tp = T(A->tstep[A->nsteps]);
        hipLaunchKernelGGL(k_ext<T>, dim3(ge), dim3(kAB), 0, s, a, psiN, arr(A->L.e1));
        hipLaunchKernelGGL(k_that<T>, dim3(ge), dim3(kAB), 0, s, a, psiN, tign_final(), tp,
                           arr(A->L.th));
        hipLaunchKernelGGL(k_adj_frac<T>, dim3(ge), dim3(kAB), 0, s, a, arr(A->L.e1),
                           arr(A->L.th), dF, c->cat, coef(), tp, arr(A->L.le), arr(A->L.e2));
        hipLaunchKernelGGL(k_adj_corners<T>, dim3(1), dim3(64), 0, s, a, arr(A->L.e1),
                           arr(A->L.le));
        const AdjFlags fl = flags();
        const int nt = ntile();
        cur = 0;
        hipLaunchKernelGGL(k_adj_ghostT<T>, dim3(gn), dim3(kAB), 0, s, a, psiN, arr(A->L.le),
                           (const T *)nullptr, (const T *)nullptr, T(0), (const T *)nullptr,
                           l1buf(0));
        hipLaunchKernelGGL(k_lt_init<T>, dim3(gn), dim3(kAB), 0, s, a, psiN, arr(A->L.e2),
                           arr(A->L.lt));
        hipLaunchKernelGGL(k_tile_any<T>, dim3(nt), dim3(kAB), 0, s, a, l1buf(0), fl.l1[0]);
        hipLaunchKernelGGL(k_tile_any<T>, dim3(nt), dim3(kAB), 0, s, a, arr(A->L.lt), fl.lt);
        // the second buffer and LP0 hold whatever the arena held: flagged, so
        // a tile that skips its work clears them
        hipLaunchKernelGGL(k_set<int32_t>, dim3(nt), dim3(kAB), 0, s, fl.l1[1], 1, (size_t)nt);
        hipLaunchKernelGGL(k_set<int32_t>, dim3(nt), dim3(kAB), 0, s, fl.lp0, 1, (size_t)nt);
        return hipGetLastError();
    }

    // Replays segment seg on the replay stream into the buffers of its
    // parity.
    hipError_t replay(int seg) {
        const int p = seg & 1;
        const int s0 = seg * A->every;
        const int s1 = s0 + A->every < A->nsteps ? s0 + A->every : A->nsteps;
        hipError_t h = hipMemcpyAsync(stack(p, 0), arr(A->L.ckpt) + (size_t)seg * n,
                                      n * sizeof(T), hipMemcpyDeviceToDevice, A->rs);
        if (h != hipSuccess) return h;
        // psi does not depend on ignition times or fuel fraction: the replay
        // recomputes psi, psi' and psi* only
        for (int k = s0; k < s1; k++) {
            h = step_raw(c, stack(p, k - s0), stack(p, k - s0 + 1), nullptr, nullptr, A->u, A->v,
                         A->tstep[k], A->dt, nullptr, nullptr, nullptr, rp0(p, k - s0),
                         rb(p, k - s0), A->rs);
            if (h != hipSuccess) return h;
        }
        return hipGetLastError();
    }

    // Reverse the steps of one replayed segment [s0, s1): part 1 of the last
    // step, then one tiled pass per step (parts 2 and 3, with part 1 of the
    // step before it except for the first step of the segment).
    hipError_t reverse_segment(int s0, int s1) {
        const int p = (s0 / A->every) & 1;
        const T *u = (const T *)A->u, *v = (const T *)A->v;
        const T *gx = (const T *)c->dzdx, *gy = (const T *)c->dzdy;
        T *LT = arr(A->L.lt), *LP0 = arr(A->L.lp0);
        double *gu = at<double>(A->L.gu), *gv = at<double>(A->L.gv), *gm = at<double>(A->L.gm);
        double *acc = at<double>(A->L.acc);
        const int32_t *set_step = at<int32_t>(A->L.set_step);
        const AdjFlags fl = flags();
        const int nt = ntile();
        AdjArgs an = a;
        an.t = A->tstep[s1 - 1];
        an.ign_active = ign_active_at(an.t);
        int k = s1 - 1 - s0;
        hipLaunchKernelGGL(k_rev_part1<T>, dim3(nt), dim3(kAB), 0, s, an, s1 - 1, set_step,
                           stack(p, k), rp0(p, k), rb(p, k), stack(p, k + 1), l1buf(cur),
                           fl.l1[cur], LT, LP0,
                           u, v, gx, gy, c->cat, coef(), ign(), dbuf(cur), acc, fl);
        for (int n_ = s1 - 1; n_ >= s0; n_--) {
            k = n_ - s0;
            an.t = A->tstep[n_];
            an.ign_active = ign_active_at(an.t);
            const int part1 = n_ > s0 ? 1 : 0;
            AdjArgs ap = a;
            ap.t = part1 ? A->tstep[n_ - 1] : an.t;
            ap.ign_active = ign_active_at(ap.t);
            hipLaunchKernelGGL(k_rev_tile<T>, dim3(nt), dim3(kRT), 0, s, an, ap, part1, n_ - 1,
                               (const T *)dbuf(cur), (const T *)l1buf(cur),
                               (const int32_t *)fl.l1[cur], (const T *)rb(p, k),
                               (const T *)rp0(p, k), (const T *)stack(p, k), LP0, l1buf(1 - cur),
                               fl.l1[1 - cur], dbuf(1 - cur), set_step,
                               part1 ? (const T *)stack(p, k - 1) : nullptr,
                               part1 ? (const T *)rp0(p, k - 1) : nullptr,
                               part1 ? (const T *)rb(p, k - 1) : nullptr, LT, u, v, gx, gy, c->cat,
                               coef(), ign(), gu, gv, gm, acc, fl);
            cur = 1 - cur;
        }
        return hipGetLastError();
    }

    int backward(const T *dF, T *grad_u, T *grad_v, double *grad_mult, double *grad_shift) {
        hipError_t h = zero_d(A->L.gu, n);
        if (h == hipSuccess) h = zero_d(A->L.gv, n);
        if (h == hipSuccess) h = zero_d(A->L.gm, n);
        if (h == hipSuccess) h = zero_d(A->L.acc, (size_t)ntile() * kShift);
        if (h == hipSuccess) h = loss_init(dF);
        // the replay stream starts after everything enqueued so far (the
        // forward's checkpoints); segment seg - 1 is replayed while seg is
        // reversed, once the reversal two segments back has freed its buffers
        if (h == hipSuccess) h = hipEventRecord(A->ev0, s);
        if (h == hipSuccess) h = hipStreamWaitEvent(A->rs, A->ev0, 0);
        if (h == hipSuccess) h = replay(A->nseg - 1);
        if (h == hipSuccess) h = hipEventRecord(A->ev_rep[(A->nseg - 1) & 1], A->rs);
        for (int seg = A->nseg - 1; seg >= 0 && h == hipSuccess; seg--) {
            const int s0 = seg * A->every;
            const int s1 = s0 + A->every < A->nsteps ? s0 + A->every : A->nsteps;
            if (seg >= 1) {
                const int q = (seg - 1) & 1;
                if (seg + 1 < A->nseg) h = hipStreamWaitEvent(A->rs, A->ev_rev[q], 0);
                if (h == hipSuccess) h = replay(seg - 1);
                if (h == hipSuccess) h = hipEventRecord(A->ev_rep[q], A->rs);
            }
            if (h == hipSuccess) h = hipStreamWaitEvent(s, A->ev_rep[seg & 1], 0);
            if (h == hipSuccess) h = reverse_segment(s0, s1);
            if (h == hipSuccess) h = hipEventRecord(A->ev_rev[seg & 1], s);
        }
        if (h != hipSuccess) return FIRE_ERR_HIP;
        // outputs
        hipLaunchKernelGGL(k_cast<T>, dim3(gn), dim3(kAB), 0, s, at<double>(A->L.gu), grad_u,
                           (int)n);
        hipLaunchKernelGGL(k_cast<T>, dim3(gn), dim3(kAB), 0, s, at<double>(A->L.gv), grad_v,
                           (int)n);
        double *part = at<double>(A->L.part), *small = at<double>(A->L.small);
        hipLaunchKernelGGL(k_cat_partial, dim3(gn), dim3(kAB), 0, s, at<double>(A->L.gm), c->cat,
                           (int)n, c->ncat, part);
        hipLaunchKernelGGL(k_col_sum, dim3(c->ncat), dim3(kAB), 0, s, part, gn, c->ncat, small);
        hipLaunchKernelGGL(k_col_sum, dim3(kShift), dim3(kAB), 0, s, at<double>(A->L.acc),
                           ntile(), kShift, small + 256);
        h = hipGetLastError();
        if (h == hipSuccess)
            h = hipMemcpyAsync(grad_mult, small, sizeof(double) * c->ncat, hipMemcpyDeviceToHost,
                               s);
        std::vector<double> sh(kShift);
        if (h == hipSuccess)
            h = hipMemcpyAsync(sh.data(), small + 256, sizeof(double) * kShift,
                               hipMemcpyDeviceToHost, s);
        if (h == hipSuccess) h = hipStreamSynchronize(s);
        if (h != hipSuccess) return FIRE_ERR_HIP;
        if (grad_shift)
            for (int g = 0; g < c->nign; g++) {
                grad_shift[2 * g] = sh[2 * g];
                grad_shift[2 * g + 1] = sh[2 * g + 1];
            }
        return FIRE_OK;
    }
};

}  // namespace

extern "C" {

size_t fire_adj_bytes(const fire_mesh *mesh, int32_t ncat, int32_t nsteps, int32_t every) {
    if (!mesh_ok(mesh) || ncat < 1 || ncat > 256 || nsteps < 1 || every < 1) return 0;
    if ((size_t)(mesh->nx + 2) * (mesh->ny + 2) > ((size_t)1 << 31)) return 0;
    return adj_layout(mesh, ncat, nsteps, every).total;
}

int fire_adj_init(fire_adj **out, fire_ctx *c, int32_t nsteps, int32_t every, void *scratch,
                  size_t scratch_bytes) {
    if (!out) return FIRE_ERR_ARG;
    *out = nullptr;
    if (!c || nsteps < 1 || every < 1 || !scratch || ((uintptr_t)scratch % kAlign) != 0)
        return FIRE_ERR_ARG;
    if (scratch_bytes < fire_adj_bytes(&c->mesh, c->ncat, nsteps, every)) return FIRE_ERR_ARG;
    fire_adj *A = new (std::nothrow) fire_adj();
    if (!A) return FIRE_ERR_OOM;
    A->c = c;
    A->nsteps = nsteps;
    A->every = every;
    A->nseg = (nsteps + every - 1) / every;
    A->arena = (char *)scratch;
    A->L = adj_layout(&c->mesh, c->ncat, nsteps, every);
    A->u = A->v = nullptr;
    A->dt = 0.0;
    A->forward_done = 0;
    A->rs = nullptr;
    A->ev0 = A->ev_rep[0] = A->ev_rep[1] = A->ev_rev[0] = A->ev_rev[1] = nullptr;
    bool ok = hipStreamCreateWithFlags(&A->rs, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&A->ev0, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < 2 && ok; k++)
        ok = hipEventCreateWithFlags(&A->ev_rep[k], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&A->ev_rev[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        fire_adj_destroy(A);
        return FIRE_ERR_HIP;
    }
    *out = A;
    return FIRE_OK;
}

int fire_adj_forward(fire_adj *A, const void *u, const void *v, double dt) {
    if (!A || !u || !v || !(dt > 0.0) || !std::isfinite(dt)) return FIRE_ERR_ARG;
    fire_ctx *c = A->c;
    const size_t n = (size_t)c->mesh.nx * c->mesh.ny;
    const size_t es = esize(&c->mesh);
    const size_t natm = (size_t)((c->mesh.nx + c->mesh.sr_x - 1) / c->mesh.sr_x) *
                        ((c->mesh.ny + c->mesh.sr_y - 1) / c->mesh.sr_y);
    A->u = u;
    A->v = v;
    A->dt = dt;
    A->forward_done = 0;
    A->tstep.assign(A->nsteps + 1, 0.0);
    A->tstep[0] = c->t;
    // set_step[i]: the step that sets node i's ignition time (-1: none does,
    // which includes nodes whose time was set before the run); the step
    // kernel stores it as it writes the time
    int32_t *set_step = reinterpret_cast<int32_t *>(A->arena + A->L.set_step);
    hipLaunchKernelGGL(k_set<int32_t>, dim3(256), dim3(kAB), 0, c->stream, set_step, -1, n);
    if (hipGetLastError() != hipSuccess) return FIRE_ERR_HIP;
    char *flux = A->arena + A->L.flux;
    int rc = FIRE_OK;
    for (int k = 0; k < A->nsteps && rc == FIRE_OK; k++) {
        if (k % A->every == 0) {
            const hipError_t h =
                hipMemcpyAsync(A->arena + A->L.ckpt + (size_t)(k / A->every) * n * es,
                               c->arena + c->off_psi[c->cur], n * es, hipMemcpyDeviceToDevice,
                               c->stream);
            if (h != hipSuccess) return FIRE_ERR_HIP;
        }
        c->mark = set_step;
        c->mark_step = k;
        rc = fire_step(c, u, v, dt, flux, flux + natm * es, nullptr);
        A->tstep[k + 1] = c->t;
    }
    c->mark = nullptr;
    c->mark_step = 0;
    if (rc != FIRE_OK) return rc;
    A->forward_done = 1;
    return FIRE_OK;
}

int fire_adj_backward(fire_adj *A, const void *dF, void *grad_u, void *grad_v, double *grad_mult,
                      double *grad_shift) {
    if (!A || !dF || !grad_u || !grad_v || !grad_mult) return FIRE_ERR_ARG;
    if (!A->forward_done || A->c->t != A->tstep[A->nsteps]) return FIRE_ERR_STATE;
    if (A->c->mesh.dtype == FIRE_F64) {
        Run<double> r(A);
        return r.backward((const double *)dF, (double *)grad_u, (double *)grad_v, grad_mult,
                          grad_shift);
    }
    Run<float> r(A);
    return r.backward((const float *)dF, (float *)grad_u, (float *)grad_v, grad_mult, grad_shift);
}

void fire_adj_destroy(fire_adj *A) {
    if (!A) return;
    if (A->rs) (void)hipStreamSynchronize(A->rs);
    for (hipEvent_t e : {A->ev0, A->ev_rep[0], A->ev_rep[1], A->ev_rev[0], A->ev_rev[1]})
        if (e) (void)hipEventDestroy(e);
    if (A->rs) (void)hipStreamDestroy(A->rs);
    delete A;
}

}  // extern "C"
