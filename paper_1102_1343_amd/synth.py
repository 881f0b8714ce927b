"""Seeded synthetic inputs for the fire-mesh time step.

This module builds inputs only: fuel-category maps, category parameter sets,
terrain gradients, surface wind fields and ignition records.  It contains none
of the method's arithmetic (no spread rate, no level set, no fuel burn), so the
HIP path and the CPU oracle can both be fed from it.

The recipes stand in for the paper's real-data cases (FireFlux, Meadow Creek,
Sect. 10), whose data are not available: they keep the fire/atmosphere
refinement ratio of 10 (Sect. 8.3), the 13 fuel categories (Sect. 2.1), a
fire-cell size of a few metres and the 6.1 m wind (Sect. 6).

Every generator takes an explicit ``numpy.random.Generator`` (PCG64) so that
a (recipe, seed) pair fixes the arrays bit for bit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Standard constants for fuel quantities the workload recipes do not draw
# (Rothermel/Anderson values for the dead fine fuel class).
FUEL_DEFAULTS = dict(
    windrf=1.0,        # a: the 6.1 m wind is used as midflame wind
    tf=0.0,            # <= 0: derive T_f from weight
    weight=1000.0,
    fgi=0.5,           # kg/m^2
    fueldepthm=0.5,    # m
    savr=8000.0,       # 1/m
    fuelmce=0.30,      # moisture of extinction
    fueldens=512.0,    # kg/m^3 (32 lb/ft^3)
    st=0.0555,
    se=0.010,
    cmbcnst=18.608e6,  # J/kg (8000 BTU/lb)
    fuelmc_g=0.08,
    ros_mult=1.0,
    ichap=0,
)

FUEL_FIELDS = tuple(FUEL_DEFAULTS.keys())
IGN_FIELDS = ("ax", "ay", "bx", "by", "t_start", "radius", "ros", "vx", "vy", "t_end")


def fuel(**kw) -> dict:
    """A fuel category record with defaults for unspecified fields."""
    f = dict(FUEL_DEFAULTS)
    for k, v in kw.items():
        if k not in f:
            raise KeyError(f"unknown fuel field {k!r}")
        f[k] = v
    return f


def ignition(ax, ay, bx=None, by=None, t_start=0.0, radius=0.0, ros=math.inf,
             vx=0.0, vy=0.0, t_end=0.0) -> dict:
    """A segment ignition a-b (a point when b is omitted), or a drip torch when
    (vx, vy) is non-zero."""
    return dict(ax=float(ax), ay=float(ay),
                bx=float(ax if bx is None else bx), by=float(ay if by is None else by),
                t_start=float(t_start), radius=float(radius), ros=float(ros),
                vx=float(vx), vy=float(vy), t_end=float(t_end))


@dataclass
class Problem:
    """Everything one fire run needs, as host arrays (float64, or float32 for
    the large single-precision workloads)."""
    nx: int
    ny: int
    dx: float
    dy: float
    sr_x: int
    sr_y: int
    fuels: list
    cat: np.ndarray            # uint8 [ny, nx]
    dzdx: np.ndarray           # [ny, nx]
    dzdy: np.ndarray
    ignitions: list
    dt: float
    steps: int
    wind: list                 # list of (u, v) [ny, nx] fields
    wind_period: int = 0       # steps per wind field (0: one field for all)
    params: dict = field(default_factory=dict)
    name: str = ""

    def wind_at(self, step: int):
        if self.wind_period <= 0 or len(self.wind) == 1:
            return self.wind[0]
        return self.wind[(step // self.wind_period) % len(self.wind)]

    def cast(self, dtype) -> "Problem":
        """Round every floating array to ``dtype`` and back to float64, so that a
        float32 run and the float64 oracle see bit-identical input values."""
        dt = np.dtype(dtype)
        r = lambda a: np.ascontiguousarray(a.astype(dt).astype(np.float64))
        return Problem(self.nx, self.ny, self.dx, self.dy, self.sr_x, self.sr_y,
                       [dict(f) for f in self.fuels], self.cat.copy(), r(self.dzdx),
                       r(self.dzdy), [dict(g) for g in self.ignitions], self.dt, self.steps,
                       [(r(u), r(v)) for (u, v) in self.wind], self.wind_period,
                       dict(self.params), self.name)


# --------------------------------------------------------------------------
# field generators
# --------------------------------------------------------------------------

def voronoi_categories(rng, nx, ny, nsites=256, ncat=13) -> np.ndarray:
    """Fuel-category map made of Voronoi patches: ``nsites`` sites uniform in
    the domain, each with a category uniform in 0..ncat-1; a cell takes the
    category of its nearest site (cell-index metric)."""
    from scipy.spatial import cKDTree

    sx = rng.uniform(0.0, nx, nsites)
    sy = rng.uniform(0.0, ny, nsites)
    scat = rng.integers(0, ncat, nsites).astype(np.uint8)
    tree = cKDTree(np.stack([sx, sy], axis=1))
    out = np.empty((ny, nx), dtype=np.uint8)
    xs = np.arange(nx) + 0.5
    rows = max(1, (1 << 22) // max(nx, 1))
    for j0 in range(0, ny, rows):
        j1 = min(ny, j0 + rows)
        yy, xx = np.meshgrid(np.arange(j0, j1) + 0.5, xs, indexing="ij")
        _, idx = tree.query(np.stack([xx.ravel(), yy.ravel()], axis=1), workers=-1)
        out[j0:j1] = scat[idx].reshape(j1 - j0, nx)
    return out


def hills_gradient(rng, nx, ny, dx, dy, nhills=8, max_slope=0.30, dtype=np.float64):
    """Analytic gradient of a sum of Gaussian hills z = sum_h A_h exp(-r^2/(2 s_h^2)).

    Centres uniform in the domain, widths s_h uniform in [0.04, 0.15] L, peak
    slopes g_h uniform in [0.05, 0.30] with A_h = g_h s_h e^(1/2) (the peak
    slope of one hill).  The summed gradient is rescaled so its largest norm
    is at most ``max_slope``.  Each hill is separable, so the fields are
    built as rank-``nhills`` products (in ``dtype``).
    """
    L = max(nx * dx, ny * dy)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    cx = rng.uniform(0, nx * dx, nhills)
    cy = rng.uniform(0, ny * dy, nhills)
    s = rng.uniform(0.04, 0.15, nhills) * L
    g = rng.uniform(0.05, 0.30, nhills)
    A = g * s * math.exp(0.5)
    ex = np.exp(-((x[None, :] - cx[:, None]) ** 2) / (2 * s[:, None] ** 2))      # [h, nx]
    ey = np.exp(-((y[None, :] - cy[:, None]) ** 2) / (2 * s[:, None] ** 2))      # [h, ny]
    fx = -(A / s ** 2)[:, None] * (x[None, :] - cx[:, None]) * ex                  # d/dx factor
    fy = -(A / s ** 2)[:, None] * (y[None, :] - cy[:, None]) * ey
    c = lambda a: np.ascontiguousarray(a, dtype=dtype)
    dzdx = c(ey.T) @ c(fx)            # [ny, nx]
    dzdy = c(fy.T) @ c(ex)
    nrm = float(np.sqrt(np.max(dzdx * dzdx + dzdy * dzdy)))
    if nrm > max_slope:
        dzdx *= dtype(max_slope / nrm)
        dzdy *= dtype(max_slope / nrm)
    return dzdx, dzdy


def fourier_wind(rng, nx, ny, dx, dy, nmodes=16, mean_speed=4.0, max_speed=8.0,
                 amp_scale=1.0, rotate_deg=0.0, dtype=np.float64):
    """Smooth surface wind: a mean wind (direction uniform, ``mean_speed``) plus
    ``nmodes`` Fourier modes alpha_m cos(2 pi k_m.x / L + phi_m) with integer
    wave vectors k_m in [-4,4]^2 minus 0 and independent amplitudes for u and
    v; the whole field is then scaled so its largest speed is ``max_speed``.
    ``amp_scale``/``rotate_deg`` perturb the result (ensemble members)."""
    Lx, Ly = nx * dx, ny * dy
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    th = rng.uniform(0, 2 * math.pi)
    k = np.zeros((nmodes, 2), dtype=np.int64)
    for m in range(nmodes):
        while True:
            kk = rng.integers(-4, 5, 2)
            if kk[0] != 0 or kk[1] != 0:
                break
        k[m] = kk
    phi = rng.uniform(0, 2 * math.pi, nmodes)
    au = rng.normal(0.0, 1.0, nmodes)
    av = rng.normal(0.0, 1.0, nmodes)
    ax_ = 2 * math.pi * k[:, 0][None, :] * x[:, None] / Lx + phi[None, :]   # [nx, m]
    by_ = 2 * math.pi * k[:, 1][None, :] * y[:, None] / Ly                  # [ny, m]
    c = lambda a: np.ascontiguousarray(a, dtype=dtype)
    X = c(np.concatenate([np.cos(ax_), np.sin(ax_)], axis=1).T)            # [2m, nx]
    Yu = c(np.concatenate([au * np.cos(by_), -au * np.sin(by_)], axis=1))   # [ny, 2m]
    Yv = c(np.concatenate([av * np.cos(by_), -av * np.sin(by_)], axis=1))
    u = Yu @ X
    u += dtype(mean_speed * math.cos(th))
    v = Yv @ X
    v += dtype(mean_speed * math.sin(th))
    sp = float(np.sqrt(np.max(u * u + v * v)))
    sc = max_speed / sp * amp_scale
    cr, sr = math.cos(math.radians(rotate_deg)), math.sin(math.radians(rotate_deg))
    if rotate_deg == 0.0:
        u *= dtype(sc)
        v *= dtype(sc)
        return u, v
    ur = dtype(sc * cr) * u - dtype(sc * sr) * v
    vr = dtype(sc * sr) * u + dtype(sc * cr) * v
    return ur, vr


def random_fuels(rng, ncat=13) -> list:
    """Category parameters drawn uniformly: load 0.1-3 kg/m^2, depth 0.1-2 m,
    moisture 0.05-0.25, surface/volume 5000-12000 1/m; burn time T_f
    log-uniform in [8, 1000] s; the rest at FUEL_DEFAULTS."""
    out = []
    for _ in range(ncat):
        out.append(fuel(
            fgi=float(rng.uniform(0.1, 3.0)),
            fueldepthm=float(rng.uniform(0.1, 2.0)),
            fuelmc_g=float(rng.uniform(0.05, 0.25)),
            savr=float(rng.uniform(5000.0, 12000.0)),
            tf=float(math.exp(rng.uniform(math.log(8.0), math.log(1000.0)))),
        ))
    return out


def line_ignitions(rng, nx, ny, dx, dy, n=4, jitter_cells=0.0):
    """``n`` line ignitions: start uniform in the central 50 % of the domain,
    random direction, length uniform in [0.02, 0.06] L, t_g uniform in
    [0, 10] s, r_g = 2 dx, S_g = 0.5 m/s."""
    L = max(nx * dx, ny * dy)
    out = []
    for _ in range(n):
        ax = rng.uniform(0.25, 0.75) * nx * dx
        ay = rng.uniform(0.25, 0.75) * ny * dy
        ang = rng.uniform(0, 2 * math.pi)
        ln = rng.uniform(0.02, 0.06) * L
        bx, by = ax + ln * math.cos(ang), ay + ln * math.sin(ang)
        if jitter_cells:
            ax += rng.uniform(-jitter_cells, jitter_cells) * dx
            ay += rng.uniform(-jitter_cells, jitter_cells) * dy
            bx += rng.uniform(-jitter_cells, jitter_cells) * dx
            by += rng.uniform(-jitter_cells, jitter_cells) * dy
        out.append(ignition(ax, ay, bx, by, t_start=float(rng.uniform(0, 10)),
                            radius=2 * dx, ros=0.5))
    return out


# --------------------------------------------------------------------------
# workload recipes
# --------------------------------------------------------------------------

SEED = 11021343


def uniform_fire(n=128, dx=6.0, steps=200, dt=0.5, wind=(2.0, 0.0)) -> Problem:
    """FP64 validation workload: n x n mesh, dx = 6 m, flat terrain, one fuel
    (load 0.5 kg/m^2, depth 0.5 m, moisture 0.08, s/v 8000 1/m, T_f = 10 s),
    constant 2 m/s wind along +x, one instantaneous circular ignition of radius
    10 m at the centre at t = 0, dt = 0.5 s, atmosphere refinement 10."""
    f = fuel(fgi=0.5, fueldepthm=0.5, fuelmc_g=0.08, savr=8000.0, tf=10.0)
    z = np.zeros((n, n))
    u = np.full((n, n), float(wind[0]))
    v = np.full((n, n), float(wind[1]))
    c = 0.5 * n * dx
    ign = [ignition(c, c, t_start=0.0, radius=10.0, ros=math.inf)]
    return Problem(n, n, dx, dx, 10, 10, [f], np.zeros((n, n), np.uint8), z, z.copy(), ign,
                   dt, steps, [(u, v)], 0,
                   dict(viscosity=0.4, viscosity_mode=0, ros_cap=math.inf,
                        boundary_policy=0, guard_width=1), name=f"uniform{n}")


def patchy_fire(n=2048, dx=6.0, steps=2000, dt=0.25, nwind=1, wind_period=0,
                seed=SEED, field_dtype=np.float64) -> Problem:
    """FP32 production workload: n x n mesh, dx = 6 m, 13 fuel categories as
    256 seeded Voronoi patches with random parameters, 8 Gaussian hills (slopes
    up to 30 %), a 16-mode Fourier wind (0-8 m/s), 4 seeded line ignitions,
    dt = 0.25 s, refinement 10, spread rate capped at 6 m/s.  With ``nwind`` > 1
    several wind fields are drawn and cycled every ``wind_period`` steps
    (time-varying coupling input).  ``field_dtype`` is the precision the
    dense fields are synthesised in (float32 for the large FP32 workloads)."""
    rng = np.random.default_rng(seed)
    fuels = random_fuels(rng)
    cat = voronoi_categories(rng, n, n)
    gzx, gzy = hills_gradient(rng, n, n, dx, dx, dtype=field_dtype)
    ign = line_ignitions(rng, n, n, dx, dx)
    winds = []
    for w in range(max(1, nwind)):
        wr = np.random.default_rng([seed, 1000 + w])
        winds.append(fourier_wind(wr, n, n, dx, dx, dtype=field_dtype))
    return Problem(n, n, dx, dx, 10, 10, fuels, cat, gzx, gzy, ign, dt, steps, winds,
                   wind_period, dict(viscosity=0.4, viscosity_mode=0, ros_cap=6.0,
                                     boundary_policy=1, guard_width=1),
                   name=f"patchy{n}")


def burning_state(prob: Problem, frac_burning=0.4, nfires=64, t0=60.0, spread=2.0,
                  seed=SEED, dtype=np.float32):
    """A mid-run state with a large burning area, to time the step where the
    fuel-fraction quadrature runs on much of the mesh: ``nfires`` discs at
    seeded centres whose union covers about ``frac_burning`` of the domain
    (radius r from Poisson coverage); psi = distance to the nearest centre
    less r within 1.5 r of a centre and 0.5 r beyond, ignition times
    t0 - (r - distance)/``spread`` inside the discs (+inf outside), F = 1
    everywhere, model time t0 (past the patchy ignitions' windows).  Returns
    (psi, tign, frac, t0) as [ny][nx] arrays."""
    rng = np.random.default_rng([seed, 99])
    W, H = prob.nx * prob.dx, prob.ny * prob.dy
    r = math.sqrt(-math.log(1.0 - frac_burning) * W * H / (nfires * math.pi))
    psi = np.full((prob.ny, prob.nx), 0.5 * r)
    for a, b in zip(rng.uniform(0.0, W, nfires), rng.uniform(0.0, H, nfires)):
        i0, i1 = max(0, int((a - 1.5 * r) / prob.dx)), min(prob.nx, int((a + 1.5 * r) / prob.dx) + 1)
        j0, j1 = max(0, int((b - 1.5 * r) / prob.dy)), min(prob.ny, int((b + 1.5 * r) / prob.dy) + 1)
        x = (np.arange(i0, i1) + 0.5) * prob.dx - a
        y = ((np.arange(j0, j1) + 0.5) * prob.dy - b)[:, None]
        psi[j0:j1, i0:i1] = np.minimum(psi[j0:j1, i0:i1], np.hypot(x[None, :], y) - r)
    tign = np.where(psi < 0, t0 + psi / spread, np.inf)
    frac = np.ones_like(psi)
    return psi.astype(dtype), tign.astype(dtype), frac.astype(dtype), float(t0)


def window(prob: Problem, i0: int, j0: int, w: int, h: int) -> Problem:
    """The sub-mesh [j0:j0+h, i0:i0+w] of ``prob`` as a problem of its own:
    arrays sliced, ignition coordinates shifted to the window origin.  With
    i0, j0 multiples of the refinement ratio its atmosphere cells are cells
    of the full mesh."""
    sl = (slice(j0, j0 + h), slice(i0, i0 + w))
    ox, oy = i0 * prob.dx, j0 * prob.dy
    c = lambda a: np.ascontiguousarray(a[sl])
    ign = [dict(g, ax=g["ax"] - ox, ay=g["ay"] - oy, bx=g["bx"] - ox, by=g["by"] - oy)
           for g in prob.ignitions]
    return Problem(w, h, prob.dx, prob.dy, prob.sr_x, prob.sr_y, [dict(f) for f in prob.fuels],
                   c(prob.cat), c(prob.dzdx), c(prob.dzdy), ign, prob.dt, prob.steps,
                   [(c(u), c(v)) for (u, v) in prob.wind], prob.wind_period, dict(prob.params),
                   f"{prob.name}[{j0}:{j0 + h},{i0}:{i0 + w}]")


def ensemble(ndom=256, side_min=256, side_max=1024, steps=500, dt=0.25, seed=SEED,
             field_dtype=np.float64) -> list:
    """Ensemble workload: ``ndom`` square domains with side uniform integer in
    [side_min, side_max], dx = 6 m, each built with the patchy-fire generators
    from a seed of its own (256 Voronoi fuel patches, 8 hills, 16-mode Fourier
    wind, 4 line ignitions); its wind amplitude scaled by U[0.8, 1.2] and
    rotated by U[-15, 15] degrees, its ignition endpoints jittered by up to 3
    cells.  All members share the 13-category fuel table of the base seed and
    the patchy-fire parameters; one wind field per member."""
    rng = np.random.default_rng([seed, 77])
    fuels = random_fuels(np.random.default_rng(seed))
    sides = rng.integers(side_min, side_max + 1, ndom)
    amp = rng.uniform(0.8, 1.2, ndom)
    rot = rng.uniform(-15.0, 15.0, ndom)
    dx = 6.0
    out = []
    for k in range(ndom):
        n = int(sides[k])
        r = np.random.default_rng([seed, 2000 + k])
        cat = voronoi_categories(r, n, n)
        gzx, gzy = hills_gradient(r, n, n, dx, dx, dtype=field_dtype)
        ign = line_ignitions(r, n, n, dx, dx, jitter_cells=3.0)
        wind = fourier_wind(r, n, n, dx, dx, amp_scale=float(amp[k]), rotate_deg=float(rot[k]),
                            dtype=field_dtype)
        out.append(Problem(n, n, dx, dx, 10, 10, [dict(f) for f in fuels], cat, gzx, gzy, ign,
                           dt, steps, [wind], 0,
                           dict(viscosity=0.4, viscosity_mode=0, ros_cap=6.0,
                                boundary_policy=1, guard_width=1),
                           name=f"ens{k}_{n}"))
    return out


def adjoint_case(n=1024, steps=500, dt=0.25, seed=SEED, field_dtype=np.float64):
    """Adjoint workload: n x n patchy landscape (13 Voronoi fuel categories,
    8 hills, 16-mode Fourier wind, dx = 6 m) with two instant circular
    ignitions of radius 3 dx at t = 0, centres uniform in the central half;
    ``steps`` steps of dt.  Returns (problem, perturbation), the perturbation
    defining the target run: multipliers U[0.8, 1.2] per category, wind x1.1,
    each centre shifted by 2 cells in a random direction."""
    rng = np.random.default_rng([seed, 5])
    dx = 6.0
    fuels = random_fuels(np.random.default_rng(seed))
    cat = voronoi_categories(rng, n, n)
    gzx, gzy = hills_gradient(rng, n, n, dx, dx, dtype=field_dtype)
    ign = []
    for _ in range(2):
        cx, cy = rng.uniform(0.3, 0.7, 2) * n * dx
        ign.append(ignition(cx, cy, t_start=0.0, radius=3 * dx, ros=math.inf))
    wind = fourier_wind(rng, n, n, dx, dx, dtype=field_dtype)
    prob = Problem(n, n, dx, dx, 10, 10, fuels, cat, gzx, gzy, ign, dt, steps, [wind], 0,
                   dict(viscosity=0.4, viscosity_mode=0, ros_cap=6.0, boundary_policy=1,
                        guard_width=1), name=f"adjoint{n}")
    ang = rng.uniform(0, 2 * math.pi, 2)
    pert = dict(mult=rng.uniform(0.8, 1.2, len(fuels)), wind_scale=1.1,
                shift=[(2 * dx * math.cos(a), 2 * dx * math.sin(a)) for a in ang])
    return prob, pert


def atmosphere(nax, nay, nz=40, dx=60.0, dy=60.0, seed=SEED, dtype=np.float64):
    """Synthetic lowest atmosphere over nax x nay columns of dx x dy metres:
    nz stretched levels (cell boundaries 0, 8, 18, 30.5, ... m, ratio 1.25,
    capped at 500 m spacing) above a terrain of 8 Gaussian hills up to 400 m,
    geopotential phi = 9.81 (z + h); roughness z0 in [0.03, 0.8] m per column
    from a smooth random field; u and v on the staggered faces following a
    log law with a horizontally varying friction velocity (16 Fourier modes,
    mean 4 m/s at 10 m) and a linear veer of up to 20 degrees over the
    column.  Returns dict(u3, v3, phi, hgt, z0)."""
    rng = np.random.default_rng([seed, 9])
    dz = np.minimum(8.0 * 1.25 ** np.arange(nz), 500.0)
    zw = np.concatenate([[0.0], np.cumsum(dz)])
    L = (nax * dx, nay * dy)
    xc = (np.arange(nax) + 0.5) * dx
    yc = (np.arange(nay) + 0.5) * dy
    hgt = np.zeros((nay, nax))
    for _ in range(8):
        cx, cy = rng.uniform(0, L[0]), rng.uniform(0, L[1])
        s = rng.uniform(0.05, 0.2) * max(L)
        hgt += rng.uniform(50, 400) * np.exp(-(((xc[None] - cx) ** 2) + ((yc[:, None] - cy) ** 2))
                                             / (2 * s * s))
    phi = 9.81 * (zw[:, None, None] + hgt[None])

    def smooth(nx_, ny_, x0, y0, amp, base):
        k = rng.integers(-3, 4, (8, 2))
        ph = rng.uniform(0, 2 * math.pi, 8)
        a = rng.normal(0, 1, 8)
        x = x0 + np.arange(nx_) * dx
        y = y0 + np.arange(ny_) * dy
        f = sum(a[m] * np.cos(2 * math.pi * (k[m, 0] * x[None] / L[0] + k[m, 1] * y[:, None] / L[1])
                              + ph[m]) for m in range(8))
        return base + amp * f / max(1e-9, np.abs(f).max())

    z0 = np.clip(smooth(nax, nay, 0.5 * dx, 0.5 * dy, 0.35, 0.4), 0.03, 0.8)
    zc = 0.5 * (zw[:-1] + zw[1:])
    th = rng.uniform(0, 2 * math.pi)
    veer = np.radians(20.0) * np.minimum(zc / zc[-1], 1.0)

    def face(nx_, ny_, x0, y0, comp):
        us = smooth(nx_, ny_, x0, y0, 1.5, 4.0)            # wind at 10 m
        prof = np.log(np.maximum(zc, 0.05) / 0.1) / math.log(10.0 / 0.1)
        ang = th + veer
        c = np.cos(ang) if comp == 0 else np.sin(ang)
        return (us[None] * (prof * c)[:, None, None]).astype(dtype)

    u3 = face(nax + 1, nay, 0.0, 0.5 * dy, 0)
    v3 = face(nax, nay + 1, 0.5 * dx, 0.0, 1)
    c = lambda a: np.ascontiguousarray(a, dtype=dtype)
    return dict(u3=c(u3), v3=c(v3), phi=c(phi), hgt=c(hgt), z0=c(z0))
