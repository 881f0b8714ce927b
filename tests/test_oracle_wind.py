"""Pins of the FP64 oracle of the coupling-input path (atmosphere wind ->
fire mesh, Sect. 6): properties the paper's definition fixes exactly."""
import math

import numpy as np

from oracle import wind as W


def _columns(nz, nay, nax, z0=0.1, h0=0.0, rng=None):
    """Stretched levels: w-level heights 0, 8, 20, 36, ... above terrain h."""
    zw = np.cumsum(np.concatenate([[0.0], 8.0 * 1.25 ** np.arange(nz)]))
    hgt = np.full((nay, nax), h0) if rng is None else rng.uniform(0, 300, (nay, nax))
    phi = W.G * (zw[:, None, None] + hgt[None])
    return phi, hgt, np.full((nay, nax), z0)


def test_cell_heights_are_level_midpoints():
    phi, hgt, _ = _columns(6, 3, 4, rng=np.random.default_rng(1))
    zc = W.cell_heights(phi, hgt)
    zw = phi / W.G - hgt[None]
    assert np.allclose(zc, 0.5 * (zw[:-1] + zw[1:]), rtol=0, atol=1e-12)
    assert np.allclose(zc[0], 4.0, atol=1e-12)


def test_log_profile_is_reproduced_exactly():
    z0 = 0.35
    z = np.array([4.0, 14.0, 28.0, 60.0, 150.0])
    A = 2.7
    vals = A * np.log(z / z0)
    for zf in (0.5, 1.0, 6.1, 9.0, 14.0, 40.0, 150.0):
        assert abs(W.log_interp(z, vals, z0, zf) - A * math.log(zf / z0)) <= 1e-12 * A * 10


def test_below_roughness_and_above_top():
    z = np.array([4.0, 14.0, 28.0])
    vals = np.array([3.0, 5.0, 6.0])
    assert W.log_interp(z, vals, 0.5, 0.5) == 0.0
    assert W.log_interp(z, vals, 0.5, 0.2) == 0.0
    assert W.log_interp(z, vals, 0.5, 500.0) == 6.0
    # a level at or below z0 is left out of the table
    z2 = np.array([0.3, 4.0, 14.0, 28.0])
    v2 = np.array([99.0, 3.0, 5.0, 6.0])
    for zf in (1.0, 6.1, 20.0):
        assert W.log_interp(z2, v2, 0.5, zf) == W.log_interp(z, vals, 0.5, zf)
    # between z0 and the first level: the log law through (z0, 0) and (z1, u1)
    zf = 2.0
    assert abs(W.log_interp(z, vals, 0.5, zf) - 3.0 * math.log(zf / 0.5) / math.log(4.0 / 0.5)) < 1e-14


def test_bilinear_hand_values():
    f = np.array([[1.0, 2.0], [3.0, 5.0]])
    assert W.bilinear(f, 0.5, 0.5) == 2.75
    assert W.bilinear(f, 1.0, 0.0) == 2.0
    assert W.bilinear(f, 0.25, 1.0) == 3.5
    assert W.bilinear(f, -3.0, 7.0) == 3.0      # clamped to the corner point
    g = np.array([[4.0, 6.0, 10.0]])             # one row: only x varies
    assert W.bilinear(g, 1.5, 0.3) == 8.0


def _linear_case(nax, nay, nz, sr_x, sr_y, dx, dy, zf, coef):
    z0 = 0.2
    phi, hgt, z0a = _columns(nz, nay, nax, z0=z0)
    zc = W.cell_heights(phi, hgt)[:, 0, 0]
    DX, DY = sr_x * dx, sr_y * dy
    a, b, c = coef
    lnz = np.log(zc / z0)
    xu = np.arange(nax + 1) * DX
    yu = (np.arange(nay) + 0.5) * DY
    u3 = (a + b * xu[None, None, :] + c * yu[None, :, None]) * lnz[:, None, None]
    xv = (np.arange(nax) + 0.5) * DX
    yv = np.arange(nay + 1) * DY
    v3 = (2 * a - c * xv[None, None, :] + b * yv[None, :, None]) * lnz[:, None, None]
    return u3, v3, phi, hgt, z0a, math.log(zf / z0)


def test_linear_fields_are_reproduced_inside():
    nax, nay, nz, sr_x, sr_y, dx, dy, zf = 5, 4, 6, 4, 3, 6.0, 5.0, 6.1
    coef = (1.5, 0.01, -0.02)
    u3, v3, phi, hgt, z0, L = _linear_case(nax, nay, nz, sr_x, sr_y, dx, dy, zf, coef)
    nx, ny = nax * sr_x, nay * sr_y
    u, v = W.fire_wind(u3, v3, phi, hgt, z0, nx, ny, sr_x, sr_y, zf=zf)
    DX, DY = sr_x * dx, sr_y * dy
    a, b, c = coef
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    # u-rows span y in [DY/2, (nay - 1/2) DY]; v-columns span x likewise
    inu = (Y >= 0.5 * DY) & (Y <= (nay - 0.5) * DY)
    inv = (X >= 0.5 * DX) & (X <= (nax - 0.5) * DX)
    assert np.max(np.abs(u - (a + b * X + c * Y) * L)[inu]) <= 1e-12
    assert np.max(np.abs(v - (2 * a - c * X + b * Y) * L)[inv]) <= 1e-12
    # outside, the clamped value of the nearest row / column
    Yc = np.clip(Y, 0.5 * DY, (nay - 0.5) * DY)
    assert np.max(np.abs(u - (a + b * X + c * Yc) * L)) <= 1e-12


def test_constant_wind_and_transposition():
    rng = np.random.default_rng(4)
    nax, nay, nz, sr_x, sr_y = 4, 3, 5, 3, 2
    phi, hgt, z0 = _columns(nz, nay, nax, rng=rng)
    z0 = rng.uniform(0.05, 0.8, (nay, nax))
    u3 = rng.normal(size=(nz, nay, nax + 1))
    v3 = rng.normal(size=(nz, nay + 1, nax))
    nx, ny = nax * sr_x - 1, nay * sr_y
    u, v = W.fire_wind(u3, v3, phi, hgt, z0, nx, ny, sr_x, sr_y)
    # swap the roles of x and y
    ut, vt = W.fire_wind(np.transpose(v3, (0, 2, 1)), np.transpose(u3, (0, 2, 1)),
                         np.transpose(phi, (0, 2, 1)), hgt.T, z0.T, ny, nx, sr_y, sr_x)
    # the same up to the order of the four bilinear terms
    assert np.allclose(ut, v.T, rtol=0, atol=1e-13) and np.allclose(vt, u.T, rtol=0, atol=1e-13)
    # a wind constant in x, y and height above z0 gives that constant at zf > z0
    zc = W.cell_heights(phi, hgt)
    assert np.all(zc > 0.8)
    c = np.full_like(u3, 3.25)
    uc, _ = W.fire_wind(c, v3, phi, hgt, np.full_like(z0, 1e-3), nx, ny, sr_x, sr_y,
                        zf=float(zc.min()) + 1.0)
    assert np.allclose(uc, 3.25, rtol=0, atol=1e-12)


def test_face_points_average_adjacent_columns():
    # two columns with different roughness and terrain: the shared face
    # (u-point I = 1) uses the mean z0 and the mean heights, the edge faces
    # their own column (reading W2)
    nz = 3
    zw = np.array([0.0, 10.0, 30.0, 70.0])
    hgt = np.array([[50.0, 80.0]])
    phi = W.G * (zw[:, None, None] + hgt[None])
    z0 = np.array([[0.1, 0.3]])
    u3 = np.zeros((nz, 1, 3))
    u3[0] = 4.0                       # first level, z1 = 5 m in both columns
    v3 = np.zeros((nz, 2, 2))
    uf, _ = W.staggered_surface_wind(u3, v3, phi, hgt, z0, 3.0)
    expect = [4.0 * math.log(3.0 / zz) / math.log(5.0 / zz) for zz in (0.1, 0.2, 0.3)]
    assert np.allclose(uf[0], expect, rtol=1e-14, atol=0)
