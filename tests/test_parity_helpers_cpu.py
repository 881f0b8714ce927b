"""The comparison helpers the GPU parity tests rely on, checked on the CPU:
the per-cell sub-cell-vertex minimum matches the whole-array one away from
the edges, a front check with no front fails, and the FP32 flux comparison
sets aside exactly the atmosphere cells that hold a knife-edge vertex."""
import numpy as np
import pytest

from paper_1102_1343_amd import synth

from parity import FluxCompare32, front_error, subpoint_min_abs, vertex_min_abs_at


def test_vertex_min_abs_matches_whole_array():
    rng = np.random.default_rng(4)
    psi = rng.normal(size=(30, 40))
    whole = subpoint_min_abs(psi)
    jj, ii = np.meshgrid(np.arange(1, 29), np.arange(1, 39), indexing="ij")
    part = vertex_min_abs_at(psi, jj.ravel(), ii.ravel())
    assert np.allclose(part, whole[1:29, 1:39].ravel(), rtol=0, atol=1e-15)


def test_front_error_refuses_an_empty_front():
    psi = np.full((16, 16), 100.0)
    with pytest.raises(AssertionError):
        front_error(psi, psi, 6.0, 6.0)
    x = (np.arange(16) - 7.5) * 6.0
    ref = np.tile(x, (16, 1))
    assert front_error(ref + 0.06, ref, 6.0, 6.0) == pytest.approx(0.01)


def test_flux_compare_sets_knife_edges_aside():
    """A cell whose node sits on psi = 0 in the oracle is a knife edge when
    the runs differ there; its own flux (from each run's F) leaves both
    per-step totals, for that step and the next."""
    import oracle
    prob = synth.uniform_fire(40, steps=1)
    tab = oracle.coef(prob.fuels)
    x = (np.arange(40) - 20.0) * 6.0 + 1.7   # no sub-cell point at psi = 0 ...
    psi_o = np.tile(x, (40, 1))
    psi_o[5, 20] = 0.0                        # ... but this node
    psi_g = psi_o.copy()
    psi_g[5, 20] = -1e-6
    frac = np.ones((40, 40))
    fs = np.zeros((4, 4))
    cmp = FluxCompare32(prob, tab)
    assert cmp.step(psi_g, psi_o, frac, frac, fs, fs, fs, fs, 0.5) == 1
    fg = frac.copy()
    fg[5, 20] = 0.9                    # only the knife cell burns in the GPU run
    dF = 0.1 / 0.5 * 36.0 * tab[0, 8]
    fs_g = np.zeros((4, 4))
    fs_g[0, 2] = dF / 3600.0           # its flux, as the atmosphere mean of a 10 x 10 cell
    psi_g2 = psi_o - 3.0               # no knife edge after this step
    n = cmp.step(psi_g2, psi_o - 3.0, fg, frac, fs_g, fs, fs, fs, 0.5)
    assert n == 1                      # the previous step's knife cell still counts
    row, full = cmp.rows[-1], cmp.full[-1]
    assert full[0] == pytest.approx(dF) and row[0] == pytest.approx(0.0, abs=1e-12 * dF)
    assert row[1] == 0.0
