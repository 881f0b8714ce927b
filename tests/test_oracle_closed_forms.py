"""Whole-step pins of the oracle against closed forms and exact identities:
planar front speed and ignition times, circle radius r0 + S t (and its
viscous modification), Heun's second order in time, exponential fuel decay,
exact heat-flux conservation, ignition arrival times, the boundary stop, and
the x/y transposition symmetry.  CPU only."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_1102_1343_amd import synth


def _problem(nx, ny, dx, dy, fuels, u=0.0, v=0.0, gzx=0.0, gzy=0.0, dt=0.25, ign=(), cat=None,
             **params):
    prm = dict(viscosity=0.4, viscosity_mode=0, ros_cap=math.inf, guard_width=1)
    prm.update(params)
    full = lambda a: np.full((ny, nx), float(a)) if np.isscalar(a) else np.asarray(a, float)
    cat = np.zeros((ny, nx), np.uint8) if cat is None else cat
    return synth.Problem(nx, ny, dx, dy, 10, 10, list(fuels), cat, full(gzx), full(gzy),
                         list(ign), dt, 0, [(full(u), full(v))], 0, prm)


def _centres(n, d):
    return (np.arange(n) + 0.5) * d


# ------------------------------------------------------------- planar front

@pytest.mark.parametrize("eps", [0.0, 0.4])
@pytest.mark.parametrize("theta_deg", [0.0, 30.0])
def test_planar_front_chaparral(eps, theta_deg):
    """psi0 = n.x - x0 with the wind along n: the front moves at exactly the
    chaparral rate S = 1.2974 U of Eq. (2) (linear psi makes the one-sided
    differences exact and the Laplacian zero, Heun is exact for constant F),
    and the ignition time of Eq. (14) is (n.x - x0)/S.  Cells within reach of
    the boundary layer at the burning edges are excluded."""
    nx, ny, dx, dy, dt, steps = 160, 96, 6.0, 5.0, 0.25, 100
    th = math.radians(theta_deg)
    U = 2.0
    prob = _problem(nx, ny, dx, dy, [synth.fuel(ichap=1)], u=U * math.cos(th),
                    v=U * math.sin(th), dt=dt, viscosity=eps)
    o = oracle.OracleFire(prob)
    X, Y = np.meshgrid(_centres(nx, dx), _centres(ny, dy))
    s = X * math.cos(th) + Y * math.sin(th)
    x0 = 480.0
    o.psi[:] = s - x0
    for _ in range(steps):
        o.step(*prob.wind[0], dt)
    S = 1.2974 * U
    t = steps * dt
    # the edge layer decays geometrically (about 3x per cell) away from the
    # burning boundaries
    mask = (X > 56 * dx) & (Y > (50 * dy if theta_deg else -1))
    assert np.max(np.abs(o.psi - (s - x0 - S * t))[mask]) <= 1e-11 * np.max(np.abs(s))
    crossed = mask & (s > x0) & (s < x0 + S * t - 1e-9)
    assert crossed.sum() > 10
    assert np.allclose(o.tign[crossed], (s[crossed] - x0) / S, rtol=1e-11, atol=1e-11)
    assert np.all(np.isinf(o.tign[mask & (s > x0 + S * t + 1e-9)]))


def test_planar_front_backing_and_slope():
    """Wind against the normal is clamped to zero (S = R0) and an uphill
    normal slope g adds d g^2 (Eq. 3), for a Rothermel fuel: the level set
    moves at the rate the coefficient form gives for that fuel."""
    nx, ny, dx, dt, steps = 120, 8, 6.0, 0.5, 60
    f = synth.fuel()
    row = oracle.coef([f])[0]
    for u, g in ((-3.0, 0.0), (0.0, 0.2), (1.5, 0.25)):
        prob = _problem(nx, ny, dx, dx, [f], u=u, gzx=g, dt=dt)
        o = oracle.OracleFire(prob)
        X, _ = np.meshgrid(_centres(nx, dx), _centres(ny, dx))
        o.psi[:] = X - 300.0
        for _ in range(steps):
            o.step(*prob.wind[0], dt)
        S = row[oracle.R0] + row[oracle.CC] * max(u, 0.0) ** row[oracle.B] + row[oracle.D] * g * g
        mask = X > 40 * dx
        assert np.allclose(o.psi[mask], (X - 300.0 - S * steps * dt)[mask], rtol=0, atol=1e-11)


# ------------------------------------------------------------- circle

def _circle_radius(dx, eps, T=60.0, r0=60.0):
    L = 300.0
    n = int(round(L / dx))
    prob = _problem(n, n, dx, dx, [synth.fuel(ichap=1, ros_mult=30.0)], dt=dx / 12, viscosity=eps)
    o = oracle.OracleFire(prob)
    x = _centres(n, dx)
    X, Y = np.meshgrid(x, x)
    c = L / 2
    o.psi[:] = np.hypot(X - c, Y - c) - r0
    for _ in range(int(round(T / prob.dt))):
        o.step(*prob.wind[0], prob.dt)
    R = []
    for row in (o.psi[n // 2], o.psi[:, n // 2]):
        i = np.where((row[:-1] <= 0) & (row[1:] > 0))[0][-1]
        xf = x[i] - row[i] * (x[i + 1] - x[i]) / (row[i + 1] - row[i])
        R.append(math.hypot(xf - c, x[n // 2] - c))
    return float(np.mean(R)), oracle.ros(o.tab[0], 0, 0)


def test_circle_radius_r0_plus_St():
    """No wind, flat terrain, uniform S = 30 * 0.03333 m/s (Eq. 2 with a
    spread multiplier): the radius tends to r0 + S t as dx -> 0, within 0.05
    fire cells already at dx = 6 m (epsilon = 0)."""
    errs = []
    for dx in (6.0, 3.0, 1.5):
        R, S = _circle_radius(dx, 0.0)
        assert S == pytest.approx(30 * 0.03333, rel=1e-14)
        errs.append(abs(R - (60.0 + S * 60.0)))
        assert errs[-1] <= 0.05 * dx
    assert errs[0] / errs[1] > 2.0 and errs[1] / errs[2] > 2.0


def test_circle_radius_with_viscosity():
    """With the viscous term eps*S*Lap~ (reading R9) a signed-distance circle
    moves at S (1 - a/R), a = eps dx, whose solution is
    R - r0 + a ln((R - a)/(r0 - a)) = S t; the computed radius converges to
    it."""
    errs = []
    for dx in (6.0, 3.0, 1.5):
        R, S = _circle_radius(dx, 0.4)
        a = 0.4 * dx
        Rm = brentq(lambda r: r - 60.0 + a * math.log((r - a) / (60.0 - a)) - S * 60.0, 61.0, 200.0)
        errs.append(abs(R - Rm))
        assert errs[-1] <= 0.15 * dx
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_heun_second_order_in_time():
    """Heun's method, Eq. (11): halving dt cuts the time error by ~4."""
    def run(dt, T=40.0):
        n, dx = 64, 6.0
        f = synth.fuel(tf=10.0)
        prob = _problem(n, n, dx, dx, [f], u=2.0, v=0.7, dt=dt)
        o = oracle.OracleFire(prob)
        X, Y = np.meshgrid(_centres(n, dx), _centres(n, dx))
        o.psi[:] = np.hypot(X - 150, Y - 160) - 40
        for _ in range(int(round(T / dt))):
            o.step(*prob.wind[0], dt)
        return o.psi.copy()
    ref = run(1 / 64)
    e = [np.abs(run(dt) - ref).max() for dt in (1.0, 0.5, 0.25)]
    assert 3.6 < e[0] / e[1] < 4.4 and 3.6 < e[1] / e[2] < 4.4, e


# ------------------------------------------------------------- fuel and flux

def test_exponential_fuel_decay_after_instant_ignition():
    """A large disc ignited at once at t = 0: every cell whose whole stencil
    burns has F(t) = exp(-t/T_f), Eq. (4)."""
    n, dx, dt, Tf = 64, 6.0, 0.5, 10.0
    c = n * dx / 2
    ign = [synth.ignition(c, c, t_start=0.0, radius=120.0)]
    prob = _problem(n, n, dx, dx, [synth.fuel(tf=Tf)], u=1.0, dt=dt, ign=ign)
    o = oracle.OracleFire(prob)
    X, Y = np.meshgrid(_centres(n, dx), _centres(n, dx))
    inner = np.hypot(X - c, Y - c) < 120.0 - 2 * dx
    for k in range(1, 41):
        o.step(*prob.wind[0], dt)
        assert np.all(o.tign[inner] == 0.0)
        assert np.allclose(o.frac[inner], math.exp(-k * dt / Tf), rtol=1e-13, atol=0)


def test_heat_flux_conservation_telescopes():
    """Sect. 4.3: the heat released into the atmosphere is exact whatever the
    quadrature error: sum_n sum_A Phi_A area_A dt = sum_cells (1 - F_end) C dx dy
    for sensible and latent heat, with partial atmosphere cells at the edges
    (96 is not a multiple of 10) and several fuels."""
    rng = np.random.default_rng(4)
    n, dx, dy, dt = 96, 6.0, 4.0, 0.25
    fuels = synth.random_fuels(rng, 4)
    cat = rng.integers(0, 4, (n, n)).astype(np.uint8)
    ign = [synth.ignition(200, 150, 300, 250, t_start=0.5, radius=12.0, ros=0.5)]
    prob = _problem(n, n, dx, dy, fuels, u=3.0, v=1.0, dt=dt, ign=ign, cat=cat, ros_cap=6.0)
    o = oracle.OracleFire(prob)
    cnt = np.zeros((10, 10))
    for J in range(10):
        for I in range(10):
            cnt[J, I] = min(10, n - 10 * J) * min(10, n - 10 * I)
    area = cnt * dx * dy
    Es = El = 0.0
    for _ in range(160):
        fs, fl = o.step(*prob.wind[0], dt)
        Es += np.sum(fs * area) * dt
        El += np.sum(fl * area) * dt
    burned = 1.0 - o.frac
    Ch = o.tab[cat, oracle.CH]
    Cq = o.tab[cat, oracle.CQ]
    Rs = np.sum(burned * Ch) * dx * dy
    Rl = np.sum(burned * Cq) * dx * dy
    assert Rs > 0 and np.sum(burned > 0.01) > 50
    assert Es == pytest.approx(Rs, rel=1e-12)
    assert El == pytest.approx(Rl, rel=1e-12)


# ------------------------------------------------------------- ignition & boundary

def test_ignition_sets_arrival_times():
    """Nodes newly covered by a growing ignition get t_g + dist/S_g (Sect. 4.4),
    which lies inside the step's window."""
    n, dx = 40, 2.0
    g = synth.ignition(37.0, 41.0, 45.0, 39.0, t_start=0.0, radius=6.0, ros=0.5)
    prob = _problem(n, n, dx, dx, [synth.fuel()], dt=1.0, ign=[g])
    o = oracle.OracleFire(prob)
    X, Y = np.meshgrid(_centres(n, dx), _centres(n, dx))
    s = np.clip(((X - 37) * 8 + (Y - 41) * -2) / 68.0, 0, 1)
    d = np.hypot(X - 37 - 8 * s, Y - 41 + 2 * s)
    for k in range(4):
        o.step(*prob.wind[0], 1.0)
        # cells first covered by psi_g at the start of step k (time k)
        newly = (d <= 0.5 * k) & (d > 0.5 * (k - 1))
        if k > 0:
            assert newly.sum() > 0
            assert np.allclose(o.tign[newly], d[newly] / 0.5, rtol=0, atol=1e-12)


def test_fire_at_boundary_sets_status():
    """Sect. 4.1: psi < 0 near the boundary ends the run."""
    n, dx = 32, 6.0
    inside = _problem(n, n, dx, dx, [synth.fuel()], dt=0.5,
                      ign=[synth.ignition(96, 96, t_start=0.0, radius=10.0)])
    o = oracle.OracleFire(inside)
    o.step(*inside.wind[0], 0.5)
    assert o.status == 0
    edge = _problem(n, n, dx, dx, [synth.fuel()], dt=0.5,
                    ign=[synth.ignition(2.0, 96, t_start=0.0, radius=10.0)])
    o = oracle.OracleFire(edge)
    o.step(*edge.wind[0], 0.5)
    assert o.status & oracle.BOUNDARY


def test_transposition_symmetry():
    """Swapping x and y (and dx/dy, u/v, the slope components, the ignition
    coordinates) transposes the result: catches mixed-up directions.  Corner
    cells are excluded (their ghost corner is built y-first, reading R19)."""
    rng = np.random.default_rng(9)
    nx, ny, dx, dy = 50, 37, 6.0, 4.5
    fuels = synth.random_fuels(rng, 3)
    cat = rng.integers(0, 3, (ny, nx)).astype(np.uint8)
    u = rng.uniform(-3, 5, (ny, nx)); v = rng.uniform(-3, 5, (ny, nx))
    gx = rng.uniform(-0.2, 0.3, (ny, nx)); gy = rng.uniform(-0.2, 0.3, (ny, nx))
    ign = [synth.ignition(120.0, 70.0, 170.0, 95.0, t_start=0.0, radius=9.0, ros=0.5)]
    a = _problem(nx, ny, dx, dy, fuels, u=u, v=v, gzx=gx, gzy=gy, dt=0.25, ign=ign, cat=cat,
                 ros_cap=6.0)
    ignT = [dict(g, ax=g["ay"], ay=g["ax"], bx=g["by"], by=g["bx"]) for g in ign]
    b = _problem(ny, nx, dy, dx, fuels, u=v.T, v=u.T, gzx=gy.T, gzy=gx.T, dt=0.25, ign=ignT,
                 cat=np.ascontiguousarray(cat.T), ros_cap=6.0)
    oa, ob = oracle.OracleFire(a), oracle.OracleFire(b)
    for _ in range(60):
        oa.step(*a.wind[0], 0.25)
        ob.step(*b.wind[0], 0.25)
    assert np.allclose(oa.psi, ob.psi.T, rtol=0, atol=1e-10)
    fin = np.isfinite(oa.tign)
    assert np.array_equal(fin, np.isfinite(ob.tign.T))
    assert np.allclose(oa.tign[fin], ob.tign.T[fin], rtol=0, atol=1e-10)
    m = np.ones_like(oa.frac, bool)
    m[[0, 0, -1, -1], [0, -1, 0, -1]] = False
    assert np.allclose(oa.frac[m], ob.frac.T[m], rtol=0, atol=1e-12)
    assert (oa.frac < 1).sum() > 20


def test_arrival_time_only_from_covering_ignitions():
    """A node newly ignited takes the earliest arrival time among the
    ignitions whose initial fire covers it (Sect. 4.4).  Here a slow drip
    torch A, radius capped at r_g = 1 m, is active but does not cover node
    (9, 12) (7.5 m away, its own arrival estimate 7.5 s); a segment B at
    x = 11.5 m started at t = 9 s with S_g = 1 m/s covers it at the step
    starting at t = 11 s, so t_i = 9 + 2/1 = 11 s, not 7.5 s."""
    n, dx = 24, 1.0
    torch = synth.ignition(2.0, 12.0, t_start=0.0, radius=1.0, ros=1.0, vx=-1e-9, vy=0.0,
                           t_end=100.0)
    seg = synth.ignition(11.5, 2.0, 11.5, 22.0, t_start=9.0, radius=5.0, ros=1.0)
    prob = _problem(n, n, dx, dx, [synth.fuel()], dt=1.0, ign=[torch, seg])
    o = oracle.OracleFire(prob, psi_init=100.0)
    for _ in range(12):
        o.step(*prob.wind[0], 1.0)
    assert o.tign[12, 9] == pytest.approx(11.0, abs=1e-12)


def test_fuel_fraction_at_the_edge_uses_ghost_time():
    """The whole domain ignited at once at t = 0: interior cells follow Eq. (4);
    edge and corner cells see ghost nodes whose ignition time is the current
    time (reading R19), which by the quadrature of Eqs. (18)-(19) gives
    F = (e^{-3/4 a} + e^{-a})/2 on an edge and
    F = (e^{-9/16 a} + 2 e^{-3/4 a} + e^{-a})/4 in a corner, a = t/T_f."""
    n, dx, dt, Tf = 20, 6.0, 0.5, 10.0
    ign = [synth.ignition(60.0, 60.0, t_start=0.0, radius=1e4)]
    prob = _problem(n, n, dx, dx, [synth.fuel(tf=Tf)], dt=dt, ign=ign)
    o = oracle.OracleFire(prob, psi_init=1e6)
    for k in range(1, 9):
        o.step(*prob.wind[0], dt)
        a = k * dt / Tf
        assert np.allclose(o.frac[1:-1, 1:-1], math.exp(-a), rtol=1e-13, atol=0)
        edge = 0.5 * (math.exp(-0.75 * a) + math.exp(-a))
        for e in (o.frac[0, 1:-1], o.frac[-1, 1:-1], o.frac[1:-1, 0], o.frac[1:-1, -1]):
            assert np.allclose(e, edge, rtol=1e-13, atol=0)
        corner = 0.25 * (math.exp(-9 / 16 * a) + 2 * math.exp(-0.75 * a) + math.exp(-a))
        for c in (o.frac[0, 0], o.frac[0, -1], o.frac[-1, 0], o.frac[-1, -1]):
            assert c == pytest.approx(corner, rel=1e-13)
