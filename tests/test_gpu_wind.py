"""Coupling input through the C ABI (needs a GPU): atmosphere wind on the
staggered faces -> surface wind on the fire mesh, against the FP64 oracle.

FP64: every fire cell within 1e-12 of the oracle (relative to the largest
speed); FP32 (inputs rounded to float32 for both sides): within 2e-6.
Shapes cover ragged fire meshes (not a multiple of the refinement), one
atmosphere row or column, one level, roughness above z_f, fire rows of
several 1024-cell chunks (refinement 1, 7, 10; a chunk spanning the most
staggered points), and the 8192 x 8192 mesh under 820 x 820 x 40
atmosphere cells on sampled cells.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import wind as W
from paper_1102_1343_amd import fire as F
from paper_1102_1343_amd import synth

from parity import host

pytestmark = pytest.mark.gpu


def _dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


def _run(atm, nx, ny, sr_x, sr_y, dt, zf=6.1):
    args = [_dev(atm[k], dt) for k in ("u3", "v3", "phi", "hgt", "z0")]
    u, v = F.wind_interp(*args, nx, ny, sr_x, sr_y, zf=zf)
    torch.cuda.synchronize()
    return host(u), host(v)


def _cast(atm, dt):
    if dt == torch.float64:
        return atm
    return {k: v.astype(np.float32).astype(np.float64) for k, v in atm.items()}


@pytest.mark.parametrize("dt,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)],
                         ids=["f64", "f32"])
@pytest.mark.parametrize("shape", [(9, 7, 10, 10, 10, 86, 70), (5, 1, 4, 3, 4, 14, 4),
                                   (1, 6, 3, 5, 2, 5, 11), (3, 3, 1, 10, 10, 30, 30),
                                   (12, 8, 20, 4, 6, 47, 45), (150, 4, 3, 10, 1, 1500, 4),
                                   (1100, 2, 2, 1, 1, 1100, 2), (1100, 2, 2, 1, 1, 1099, 2),
                                   (300, 3, 2, 7, 1, 2050, 3)],
                         ids=["9x7x10", "row", "column", "one-level", "ragged", "wide-sr10",
                              "wide-sr1", "wide-sr1-ragged", "wide-sr7"])
def test_wind_matches_oracle(dt, tol, shape):
    nax, nay, nz, sr_x, sr_y, nx, ny = shape
    atm = synth.atmosphere(nax, nay, nz=nz, dx=6.0 * sr_x, dy=6.0 * sr_y, seed=nax * 100 + nay)
    ref = _cast(atm, dt)
    u_o, v_o = W.fire_wind(ref["u3"], ref["v3"], ref["phi"], ref["hgt"], ref["z0"], nx, ny,
                           sr_x, sr_y)
    u_g, v_g = _run(atm, nx, ny, sr_x, sr_y, dt)
    scale = max(np.abs(u_o).max(), np.abs(v_o).max())
    assert scale > 0.5
    assert np.max(np.abs(u_g - u_o)) <= tol * scale
    assert np.max(np.abs(v_g - v_o)) <= tol * scale


def test_roughness_above_zf_gives_zero_and_high_zf_the_top_value():
    atm = synth.atmosphere(6, 5, nz=8, dx=60.0, dy=60.0, seed=3)
    atm = dict(atm)
    z0 = atm["z0"].copy()
    z0[2, 3] = 50.0                      # above z_f: the faces of this column drop
    atm["z0"] = z0
    u_o, v_o = W.fire_wind(atm["u3"], atm["v3"], atm["phi"], atm["hgt"], atm["z0"], 60, 50, 10,
                           10)
    u_g, v_g = _run(atm, 60, 50, 10, 10, torch.float64)
    assert np.max(np.abs(u_g - u_o)) <= 1e-12 * np.abs(u_o).max()
    assert np.max(np.abs(v_g - v_o)) <= 1e-12 * np.abs(v_o).max()
    # the faces of that column have z0 > z_f: their wind is 0
    uf, vf = W.staggered_surface_wind(atm["u3"], atm["v3"], atm["phi"], atm["hgt"], atm["z0"],
                                      6.1)
    assert uf[2, 3] == 0.0 and uf[2, 4] == 0.0 and vf[2, 3] == 0.0 and vf[3, 3] == 0.0
    hi = _run(atm, 60, 50, 10, 10, torch.float64, zf=1e5)
    uo_hi, _ = W.fire_wind(atm["u3"], atm["v3"], atm["phi"], atm["hgt"], atm["z0"], 60, 50, 10,
                           10, zf=1e5)
    assert np.max(np.abs(hi[0] - uo_hi)) <= 1e-12 * np.abs(uo_hi).max()


def test_wind_8192_sampled():
    nax = nay = 820
    atm = synth.atmosphere(nax, nay, nz=40, dx=60.0, dy=60.0, dtype=np.float32)
    u_g, v_g = _run(atm, 8192, 8192, 10, 10, torch.float32)
    ref = _cast(atm, torch.float32)
    rng = np.random.default_rng(11)
    pts = [(0, 0), (8191, 8191), (0, 8191), (8191, 0), (4096, 17)]
    pts += [tuple(p) for p in rng.integers(0, 8192, (60, 2))]
    err = 0.0
    scale = 0.0
    for i, j in pts:
        uo, vo = W.fire_wind_sample(ref["u3"], ref["v3"], ref["phi"], ref["hgt"], ref["z0"], i,
                                    j, 10, 10)
        err = max(err, abs(u_g[j, i] - uo), abs(v_g[j, i] - vo))
        scale = max(scale, abs(uo), abs(vo))
    assert scale > 1.0
    assert err <= 2e-6 * scale
    assert np.isfinite(u_g).all() and np.isfinite(v_g).all()
