// Device arithmetic shared by the step kernels and the reverse (adjoint)
// kernels of the fire-mesh time step: the math wrappers, the spread rate of
// Eq. (3), the boundary extrapolation of Sect. 4.1, the right-hand side of
// Eqs. (12)-(13) at one node and the ignition geometry of Sect. 4.4.  Both
// sides call these same functions, so a recomputed forward quantity is the
// forward's value bit for bit.
#pragma once

#include "fire_internal.h"

#include <cmath>

namespace fire {
namespace dev {

// ---------------------------------------------------------------- math
template <typename T> struct M;

template <> struct M<float> {
    // x >= 0; x = 0 gives 0 for b > 0
    static __device__ __forceinline__ float powp(float x, float b) {
        return __builtin_amdgcn_exp2f(b * __builtin_amdgcn_logf(x));
    }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float div(float a, float b) {
        return a * __builtin_amdgcn_rcpf(b);
    }
    // 1 - exp(-x); its absolute rounding error is that of F itself
    static __device__ __forceinline__ float one_m_exp_neg(float x) {
        return 1.0f - __builtin_amdgcn_exp2f(-1.4426950408889634f * x);
    }
    static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
};

template <> struct M<double> {
    static __device__ __forceinline__ double powp(double x, double b) { return ::pow(x, b); }
    static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double one_m_exp_neg(double x) { return -::expm1(-x); }
    static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
};

// max / min / |.| as single instructions (for non-NaN operands the same as
// the comparisons they replace; a NaN operand yields the other one)
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float vabs(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double vabs(double a) { return __builtin_fabs(a); }
template <typename T> __device__ __forceinline__ bool is_inf(T a) { return a == M<T>::inf(); }
// median of three for lo <= hi: min(max(x, lo), hi) in one instruction
__device__ __forceinline__ float med3(float x, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(x, lo, hi);
}
__device__ __forceinline__ double med3(double x, double lo, double hi) {
    return vmin(vmax(x, lo), hi);
}

// Spread rate, Eq. (3), with the category multiplier and the cap:
// S = min{cap, m max{S0, R0 + c min{e, max{0,U}}^b + d max{0, tan phi}^2}}.
template <typename T>
__device__ __forceinline__ T ros(const T *row, T un, T tn, T cap) {
    const T U = vmin(vmax(un, T(0)), row[kE]);
    const T g = vmax(tn, T(0));
    T s = row[kR0] + row[kC] * M<T>::powp(U, row[kB]) + row[kD] * g * g;
    s = vmax(s, row[kS0]);
    return vmin(row[kM] * s, cap);
}

// Boundary extrapolation of Sect. 4.1: never below either source node.
template <typename T> __device__ __forceinline__ T ghost(T pb, T pb1) {
    return vmax(pb + (pb - pb1), vmax(pb, pb1));
}

template <typename T> struct Consts {
    T rdx, rdy, eps, cap;
    int visc_mode;
};

// Per-category row of the in-LDS table, the multiplier m_k folded in
// (m max{S0, R0 + c U^b + d g^2} = max{m S0, m R0 + m c U^b + m d g^2}, m >= 0).
enum { kLR0, kLC, kLD, kLB, kLE, kLS0, kLTf, kLCh, kLCq, kLPad0, kLPad1, kLPad2, kLRow };

template <typename T> struct alignas(4 * sizeof(T)) V4 { T x, y, z, w; };

// Table row of one category from its coefficient-table entry g.
// The floor is stored as min(m S0, cap) so that the floor and the cap of
// Eq. (3) are one median: min(max(s, m S0), cap) = med3(s, min(m S0, cap), cap).
template <typename T> __device__ __forceinline__ void make_row(const T *g, T *r, T cap) {
    const T m = g[kM];
    r[kLR0] = m * g[kR0];
    r[kLC] = m * g[kC];
    r[kLD] = m * g[kD];
    r[kLB] = g[kB];
    r[kLE] = g[kE];
    r[kLS0] = vmin(m * g[kS0], cap);
    r[kLTf] = T(1) / g[kTf];
    r[kLCh] = g[kCh];
    r[kLCq] = g[kCq];
    r[kLPad0] = r[kLPad1] = r[kLPad2] = T(0);
}

// An object in LDS, addressed with 32-bit offsets.
template <typename T> using lds_t = T __attribute__((address_space(3)));

// Spread rate, Eq. (3), with multiplier and cap, from a table row (r0, r1:
// its first eight entries).
template <typename T>
__device__ __forceinline__ T ros_v4(const V4<T> &r0, const V4<T> &r1, T un, T tn, T cap) {
    const T U = med3(un, T(0), r1.x);
    const T g = vmax(tn, T(0));
    const T s = r0.x + r0.y * M<T>::powp(U, r0.w) + r0.z * (g * g);
    return med3(s, r1.y, cap);
}
template <typename T>
__device__ __forceinline__ T ros_row(const T *row, T un, T tn, T cap) {
    return ros_v4(*reinterpret_cast<const V4<T> *>(row),          // R0 c d b
                  *reinterpret_cast<const V4<T> *>(row + 4),      // e min(S0,cap) Tf Ch
                  un, tn, cap);
}
template <typename T>
__device__ __forceinline__ T ros_row(const lds_t<T> *row, T un, T tn, T cap) {
    const lds_t<V4<T>> *q = reinterpret_cast<const lds_t<V4<T>> *>(row);
    V4<T> r0, r1;
    r0.x = q[0].x; r0.y = q[0].y; r0.z = q[0].z; r0.w = q[0].w;
    r1.x = q[1].x; r1.y = q[1].y; r1.z = q[1].z; r1.w = q[1].w;
    return ros_v4(r0, r1, un, tn, cap);
}

// Right-hand side of Eq. (12) at a node from its value pc and its four
// neighbours (west, east, south, north).  The Godunov choice of Eq. (13)
// enters only through its square, which for every sign pattern is
// max(max(D-,0)^2, min(D+,0)^2); the dx-scaled Laplacian is (D+ - D-) summed
// over x and y.  The central gradient is taken as (psi_E - psi_W)/dx (its
// factor 1/2 cancels in the normal) straight from the two nodes, so it is
// exactly zero when they are equal -- as at a domain corner whose ghosts
// mirror the inner nodes -- whatever the compiler fuses.
template <typename T, typename RowPtr>
__device__ __forceinline__ T rhs5(T pc, T pw, T pe, T ps, T pn, T u, T v, T gzx, T gzy,
                                  RowPtr row, const Consts<T> &c) {
    const T dmx = (pc - pw) * c.rdx, dpx = (pe - pc) * c.rdx;
    const T dmy = (pc - ps) * c.rdy, dpy = (pn - pc) * c.rdy;
    // max(max(D-,0)^2, min(D+,0)^2) = max(D-, -D+, 0)^2 exactly
    const T gx = vmax(vmax(dmx, -dpx), T(0)), gy = vmax(vmax(dmy, -dpy), T(0));
    const T up = M<T>::sqrt(gx * gx + gy * gy);
    const T cx = (pe - pw) * c.rdx, cy = (pn - ps) * c.rdy;
    const T cn2 = cx * cx + cy * cy;
    const T inv = cn2 > T(0) ? M<T>::rsqrt(cn2) : T(0);
    const T nx = cx * inv, ny = cy * inv;
    const T S = ros_row(row, u * nx + v * ny, gzx * nx + gzy * ny, c.cap);
    const T lap = (dpx - dmx) + (dpy - dmy);
    const T visc = c.visc_mode == 0 ? c.eps * S * lap : c.eps * lap;
    return visc - S * up;
}

// Fused multiply-add as one rounding, whatever the compiler's contraction
// setting: the ignition geometry below is evaluated by the step kernels and
// by the reverse kernels, which must take exactly the forward's values.
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One ignition's geometry at time t (IgnGeo): plain IEEE operations with no
// contraction into fused multiply-adds, so every kernel that forms it (the
// per-step table of the step kernels, the reverse kernels) gets the same
// bits.
template <typename T>
__device__ __forceinline__ bool ign_setup(const fire_ignition &g, double t, IgnGeo<T> &o) {
#pragma clang fp contract(off)
    const bool torch = (g.vx != 0.0 || g.vy != 0.0);
    const double tend = torch ? g.t_end : g.t_start;
    const bool inst = __builtin_isinf(g.ros);
    const double grow = inst ? 0.0 : g.radius / g.ros;
    if (!(t >= g.t_start && t <= tend + grow)) return false;
    double bx = g.bx, by = g.by;
    if (torch) {
        const double te = t < g.t_end ? t : g.t_end;
        bx = g.ax + g.vx * (te - g.t_start);
        by = g.ay + g.vy * (te - g.t_start);
    }
    const double ex = bx - g.ax, ey = by - g.ay;
    const double L2 = ex * ex + ey * ey;
    const double r = g.ros * (t - g.t_start);
    o.ax = g.ax;
    o.ay = g.ay;
    o.ex = T(ex);
    o.ey = T(ey);
    o.exL = L2 > 0.0 ? T(ex / L2) : T(0);
    o.eyL = L2 > 0.0 ? T(ey / L2) : T(0);
    o.rad = T(inst ? g.radius : (r < g.radius ? r : g.radius));
    o.tg = T(g.t_start);
    o.lenv = torch ? T(::sqrt(L2) / ::sqrt(g.vx * g.vx + g.vy * g.vy)) : T(0);
    o.invS = inst ? T(0) : T(1.0 / g.ros);
    o.t = T(t);
    o.pad = T(0);
    return true;
}

// Offsets of a node centre from the segment start, formed in double from
// global coordinates and rounded once: px from the node's column, py from
// its row, and the row's share of the projection parameter, by = py eyL.
template <typename T>
__device__ __forceinline__ T ign_px(const IgnGeo<T> &g, int gx, double dx) {
    return T(((double)gx + 0.5) * dx - g.ax);
}
template <typename T>
__device__ __forceinline__ T ign_py(const IgnGeo<T> &g, int gy, double dy) {
    return T(((double)gy + 0.5) * dy - g.ay);
}
template <typename T> __device__ __forceinline__ T ign_by(const IgnGeo<T> &g, T py) {
    return py * g.eyL;
}

// Nearest point of the segment (Eq. 20): parameter s in [0, 1], the offset
// (qx, qy) from it and its square d2.
template <typename T> struct IgnNear {
    T s, qx, qy, d2;
};
template <typename T>
__device__ __forceinline__ IgnNear<T> ign_near(const IgnGeo<T> &g, T px, T py, T by) {
    IgnNear<T> r;
    r.s = med3(fmaT(px, g.exL, by), T(0), T(1));
    r.qx = fmaT(-r.s, g.ex, px);
    r.qy = fmaT(-r.s, g.ey, py);
    r.d2 = fmaT(r.qx, r.qx, r.qy * r.qy);
    return r;
}

// Arrival time of the initial fire at the node (drip-torch form), capped at t.
template <typename T>
__device__ __forceinline__ T ign_arrival(const IgnGeo<T> &g, const IgnNear<T> &q, T d) {
    return vmin(fmaT(d, g.invS, fmaT(q.s, g.lenv, g.tg)), g.t);
}

// 1 + a margin above the relative rounding of d2, of its square root and of
// (p + r)^2: d2 > (p + r)^2 (1 + margin) proves sqrt(d2) - r >= p after
// rounding.
template <typename T> struct IgnMargin;
template <> struct IgnMargin<float> {
    static __device__ __forceinline__ float v() { return 1.0f + 0x1p-19f; }
};
template <> struct IgnMargin<double> {
    static __device__ __forceinline__ double v() { return 1.0 + 0x1p-40; }
};

// The same as ign_apply where psi_g > 0 is known for the node (a tile whose
// lower bound of psi_g is positive): only p can change.
template <typename T>
__device__ __forceinline__ void ign_lower(const IgnGeo<T> &g, T px, T py, T by, T &p) {
    const IgnNear<T> q = ign_near(g, px, py, by);
    if (sizeof(T) == 8) {
        const T pr = p + g.rad;
        if (p > T(0) && q.d2 > pr * pr * IgnMargin<T>::v()) return;
    }
    const T pg = M<T>::sqrt(q.d2) - g.rad;
    p = pg < p ? pg : p;   // a NaN p stays NaN
}

// Applies one ignition to node value p (Eq. 21): p := min(p, psi_g), with
// psi_g = d - r_g of Eq. (20), and a node with psi_g <= 0 offers its arrival
// time to tig (the minimum over ignitions).  FP32 evaluates every node
// without branches (the square root costs less than the test that would
// skip it); FP64, whose square root is a long sequence, skips it where p > 0
// and d2 alone shows psi_g >= p (so also psi_g > 0): neither can change
// there, so the result is the same as without the test.  Returns bit 0 if p
// was lowered, bit 1 if tig was.
template <typename T>
__device__ __forceinline__ int ign_apply(const IgnGeo<T> &g, T px, T py, T by, T &p, T &tig) {
    const IgnNear<T> q = ign_near(g, px, py, by);
    if (sizeof(T) == 8) {
        const T pr = p + g.rad;
        if (p > T(0) && q.d2 > pr * pr * IgnMargin<T>::v()) return 0;
    }
    const T d = M<T>::sqrt(q.d2);
    const T pg = d - g.rad;
    const T a = ign_arrival(g, q, d);
    const bool lit = pg <= T(0) && a < tig;
    const bool lower = pg < p;   // a NaN p stays NaN (reported by the status word)
    tig = lit ? a : tig;
    p = lower ? pg : p;
    return (lit ? 2 : 0) | (lower ? 1 : 0);
}

}  // namespace dev
}  // namespace fire
