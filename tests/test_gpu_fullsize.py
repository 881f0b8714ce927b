"""Parity at the production sizes, in the launch configuration bench.py times
(needs a GPU).

8192 x 8192 FP32 patchy workload (default tile), against the FP64 oracle on
the FP32-rounded inputs:
  * the whole mesh for the first 50 steps (all four ignitions start within
    them): total sensible and latent heat flux over the domain within 1e-4
    relative per step (once above 1e-3 of its peak; fire cells where a
    sub-cell vertex of the oracle sits within the runs' local psi discrepancy
    of the Eq. (17) switch are left out of that step, see
    parity.FluxCompare32) and summed over the steps (every cell), front
    position within 0.05 cell everywhere, F where no front is near;
  * after 120 steps, windows of 700 x 700 around the start and around the
    end of each ignition segment (every window has burning cells in its
    compared interior).  psi at a node after n steps depends only on psi^0
    within 2n cells (two Heun stages of one cell each) and F on one more, so
    on the window interior 2n + 3 cells from the edge the oracle's values are
    the full mesh's: front position and F are compared there.

2048 x 2048 FP32 patchy workload over its full 2000 steps: front position
every 100 steps, total fluxes every step and integrated over the run, as
above (the check on FP32 cancellation in F^n - F^{n+1} over long burns with
burn times up to 1000 s).  It takes several minutes of oracle time on the
host, so it runs only when FIRE_LONG_TESTS is set.
F is stored in FP32, so one cell's change over a step carries up to ~6e-8 of
rounding; the flux bar is met on domain totals, not on fires of a few cells.

2048 x 2048 FP64 patchy workload: the whole field against the oracle for the
first 50 steps (ignitions active) to the FP64 bar.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1102_1343_amd import synth

from parity import Compare64, FluxCompare32, front_error, gpu_fire, host, total_flux

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def big():
    _log("generating patchy8192")
    return synth.patchy_fire(n=8192, steps=1000, nwind=4, wind_period=10, field_dtype=np.float32)


def _gpu_run(prob, steps):
    W = [(torch.from_numpy(np.ascontiguousarray(u)).cuda(),
          torch.from_numpy(np.ascontiguousarray(v)).cuda()) for u, v in prob.wind]
    g = gpu_fire(prob, torch.float32)
    assert g.get_tile() == (120, 20)
    fs, fl = g.new_flux()
    tot = []
    for k in range(steps):
        u, v = W[(k // prob.wind_period) % len(W)]
        g.step(u, v, prob.dt, fs, fl)
        tot.append((total_flux(host(fs), prob), total_flux(host(fl), prob)))
    torch.cuda.synchronize()
    return g, np.array(tot)


def test_fullsize_8192_fp32_whole_domain(big):
    prob = big
    steps = 50
    W = [(torch.from_numpy(np.ascontiguousarray(u)).cuda(),
          torch.from_numpy(np.ascontiguousarray(v)).cuda()) for u, v in prob.wind]
    g = gpu_fire(prob, torch.float32)
    assert g.get_tile() == (120, 20)
    fs, fl = g.new_flux()
    p64 = prob.cast(np.float32)
    o = oracle.OracleFire(p64)
    cmp = FluxCompare32(prob, o.tab)
    for k in range(steps):
        u, v = W[(k // prob.wind_period) % len(W)]
        g.step(u, v, prob.dt, fs, fl)
        fs_o, fl_o = o.step(*p64.wind_at(k), prob.dt)
        cmp.step(host(g.psi), o.psi, host(g.frac), o.frac, host(fs), host(fl), fs_o, fl_o,
                 prob.dt)
    psi_g, frac_g = host(g.psi), host(g.frac)
    _log(f"{steps} steps done, status {g.status()}, burning cells {(o.psi < 0).sum()}")
    cmp.check("8192^2", _log)
    err = front_error(psi_g, o.psi, prob.dx, prob.dy)
    _log(f"front error {err:.2e} cells")
    assert err <= 0.05
    far = np.abs(o.psi) > 2 * prob.dx
    assert np.max(np.abs(frac_g - o.frac)[far]) <= 1e-4
    assert (o.frac < 1).sum() > 1000


def test_fullsize_8192_fp32_windows(big):
    prob = big
    steps = 120
    g, _ = _gpu_run(prob, steps)
    psi_g, tig_g, frac_g = host(g.psi), host(g.tign), host(g.frac)
    centres = [(ig["ax"], ig["ay"]) for ig in prob.ignitions]
    centres += [(ig["bx"], ig["by"]) for ig in prob.ignitions[:2]]
    w = 700
    m = 2 * steps + 3
    psi0 = math.hypot(prob.nx * prob.dx, prob.ny * prob.dy)
    for cx, cy in centres:
        i0 = int(min(max(0, cx / prob.dx - w / 2), prob.nx - w)) // 10 * 10
        j0 = int(min(max(0, cy / prob.dy - w / 2), prob.ny - w)) // 10 * 10
        win = synth.window(prob, i0, j0, w, w).cast(np.float32)
        o = oracle.OracleFire(win, psi_init=psi0)
        for k in range(steps):
            o.step(*win.wind_at(k), prob.dt)
        sl = (slice(j0 + m, j0 + w - m), slice(i0 + m, i0 + w - m))
        osl = (slice(m, w - m), slice(m, w - m))
        err = front_error(psi_g[sl], o.psi[osl], prob.dx, prob.dy)
        burning = int((o.psi[osl] < 0).sum())
        _log(f"window ({i0},{j0}): front error {err:.2e} cells, burning {burning}")
        assert burning > 100
        assert err <= 0.05
        far = np.abs(o.psi[osl]) > 2 * prob.dx
        assert np.max(np.abs(frac_g[sl] - o.frac[osl])[far]) <= 1e-4
        # ignition times agree (to a sanity bound; FP32 crossing times scale
        # with psi's rounding over the spread rate) where no front is near
        fin = np.isfinite(tig_g[sl]) & np.isfinite(o.tign[osl])
        assert np.array_equal(np.isfinite(tig_g[sl]) & far, np.isfinite(o.tign[osl]) & far)
        if fin.any():
            assert np.max(np.abs(tig_g[sl][fin] - o.tign[osl][fin])) <= 0.1


def test_patchy2048_fp64_full_field():
    prob = synth.patchy_fire(n=2048, steps=50)
    _log("fp64 parity patchy2048, 50 steps, whole field")
    g = gpu_fire(prob, torch.float64)
    o = oracle.OracleFire(prob)
    u = torch.from_numpy(prob.wind[0][0]).cuda()
    v = torch.from_numpy(prob.wind[0][1]).cuda()
    cmp = Compare64(prob)
    fs, fl = g.new_flux()
    for k in range(prob.steps):
        prev, t_prev = o.psi.copy(), o.t
        g.step(u, v, prob.dt, fs, fl)
        fs_o, fl_o = o.step(*prob.wind[0], prob.dt)
        torch.cuda.synchronize()
        cmp.step(g, o, fs, fl, fs_o, fl_o, prev, t_prev)
    assert np.isfinite(o.tign).sum() > 100


@pytest.mark.skipif(not os.environ.get("FIRE_LONG_TESTS"),
                    reason="runs the FP64 oracle for 2000 steps of 2048 x 2048 (several "
                           "minutes of host time); set FIRE_LONG_TESTS=1 to run it")
def test_fullsize_2048_fp32_full_length(capsys):
    prob = synth.patchy_fire(n=2048, steps=2000, field_dtype=np.float32)
    steps = prob.steps

    def _log(msg):   # progress past pytest's capture: the run is long
        with capsys.disabled():
            print(msg, flush=True)

    _log(f"fp32 patchy2048, {steps} steps, GPU and oracle ({oracle.threads()} threads) "
         "in lockstep")
    u = torch.from_numpy(np.ascontiguousarray(prob.wind[0][0])).cuda()
    v = torch.from_numpy(np.ascontiguousarray(prob.wind[0][1])).cuda()
    g = gpu_fire(prob, torch.float32)
    fs, fl = g.new_flux()
    p64 = prob.cast(np.float32)
    o = oracle.OracleFire(p64)
    cmp = FluxCompare32(prob, o.tab)
    for k in range(steps):
        g.step(u, v, prob.dt, fs, fl)
        fs_o, fl_o = o.step(*p64.wind_at(k), prob.dt)
        psi_g = host(g.psi)
        cmp.step(psi_g, o.psi, host(g.frac), o.frac, host(fs), host(fl), fs_o, fl_o, prob.dt)
        if (k + 1) % 100 == 0:
            err = front_error(psi_g, o.psi, prob.dx, prob.dy)
            _log(f"step {k + 1}: front error {err:.2e} cells, burning {(o.psi < 0).sum()}")
            assert err <= 0.05
    cmp.check("2048^2 x 2000", _log)
    assert (o.frac < 0.5).sum() > 1000
