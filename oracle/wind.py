"""FP64 oracle of the coupling-input path: atmosphere wind -> fire mesh.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of bench.py, never by the product path.

Follows the coupling section of the paper (Sect. 6): the wind is brought to
the height z_f above the terrain (6.1 m) assuming the logarithmic profile,
by piecewise-linear interpolation in ln z through (ln z0, 0) and the values
at the heights of the atmospheric cell centres, which come from the
geopotential; u and v are then each interpolated bilinearly from their
staggered points (midpoints of the cell faces, Fig. 1) to the centres of the
fire cells.

Readings (where the paper does not say):
  W1 heights of the cell centres: z_k = (phi_k + phi_{k+1}) / (2 g) - h, with
     phi at the levels bounding the cell and h the terrain height;
  W2 under a u-point (v-point) the column heights and z0 are the mean of the
     two adjacent columns, or the one column at the domain edge;
  W3 levels with z_k <= z0 are left out; above the highest level the top
     value is kept; z_f <= z0 gives 0;
  W4 bilinear weights from the point positions, coordinates clamped to the
     extent of the staggered points (constant beyond the outermost ones).

Parity status: pinned (tests/test_oracle_wind.py): exact log profiles,
z_f <= z0, linear horizontal fields, constants, x/y transposition.
"""
from __future__ import annotations

import math

import numpy as np

G = 9.81


def cell_heights(phi, hgt, g=G):
    """W1: heights above the terrain of the cell centres, [nz][nay][nax]."""
    phi = np.asarray(phi, dtype=np.float64)
    return 0.5 * (phi[:-1] + phi[1:]) / g - np.asarray(hgt, dtype=np.float64)[None]


def log_interp(z, val, z0, zf):
    """Value at zf of the piecewise-linear interpolant in ln z of
    (ln z0, 0), (ln z_k, val_k) over the levels with z_k > z0 (W3)."""
    if not zf > z0:
        return 0.0
    keep = [(zk, vk) for zk, vk in zip(z, val) if zk > z0]
    xs = [math.log(z0)] + [math.log(zk) for zk, _ in keep]
    ys = [0.0] + [float(vk) for _, vk in keep]
    # np.interp keeps the end values outside the table (top value above)
    return float(np.interp(math.log(zf), xs, ys))


def u_point(u3, zc, z0, I, J, zf):
    """u at height zf under u-point (I, J) (W2, W3); zc from cell_heights."""
    nax = zc.shape[2]
    cl, cr = max(I - 1, 0), min(I, nax - 1)
    z = 0.5 * (zc[:, J, cl] + zc[:, J, cr])
    return log_interp(z, u3[:, J, I], 0.5 * (z0[J, cl] + z0[J, cr]), zf)


def v_point(v3, zc, z0, I, J, zf):
    """v at height zf under v-point (I, J)."""
    nay = zc.shape[1]
    cb, ct = max(J - 1, 0), min(J, nay - 1)
    z = 0.5 * (zc[:, cb, I] + zc[:, ct, I])
    return log_interp(z, v3[:, J, I], 0.5 * (z0[cb, I] + z0[ct, I]), zf)


def staggered_surface_wind(u3, v3, phi, hgt, z0, zf, g=G):
    """u at the u-points [nay][nax+1] and v at the v-points [nay+1][nax] at
    height zf (W1-W3)."""
    u3 = np.asarray(u3, dtype=np.float64)
    v3 = np.asarray(v3, dtype=np.float64)
    z0 = np.asarray(z0, dtype=np.float64)
    zc = cell_heights(phi, hgt, g)
    nz, nay, nax = zc.shape
    uf = np.zeros((nay, nax + 1))
    vf = np.zeros((nay + 1, nax))
    for J in range(nay):
        for I in range(nax + 1):
            uf[J, I] = u_point(u3, zc, z0, I, J, zf)
    for J in range(nay + 1):
        for I in range(nax):
            vf[J, I] = v_point(v3, zc, z0, I, J, zf)
    return uf, vf


def bilinear(f, px, py):
    """Bilinear value of the 2-D point field f[J][I] (I along x) at the
    fractional point coordinates (px, py), each clamped to the field (W4)."""
    f = np.asarray(f)
    return bilinear_fn(lambda J, I: f[J, I], f.shape[1], f.shape[0], px, py)


def bilinear_fn(get, nx, ny, px, py):
    """bilinear() on a field of nx x ny points given by get(J, I)."""
    px = min(max(px, 0.0), nx - 1.0)
    py = min(max(py, 0.0), ny - 1.0)
    i0 = min(int(math.floor(px)), max(nx - 2, 0))
    j0 = min(int(math.floor(py)), max(ny - 2, 0))
    i1, j1 = min(i0 + 1, nx - 1), min(j0 + 1, ny - 1)
    tx, ty = px - i0, py - j0
    return ((1 - tx) * (1 - ty) * get(j0, i0) + tx * (1 - ty) * get(j0, i1)
            + (1 - tx) * ty * get(j1, i0) + tx * ty * get(j1, i1))


def fire_wind_at(uf, vf, i, j, sr_x, sr_y):
    """(u, v) at the centre of fire cell (i, j).  With atmosphere cells of
    sr_x x sr_y fire cells, a fire centre sits at x / DX = (i + 1/2) / sr_x;
    u-points are at x / DX = I, y / DY = J + 1/2, v-points at
    x / DX = I + 1/2, y / DY = J."""
    X = (i + 0.5) / sr_x
    Y = (j + 0.5) / sr_y
    return bilinear(uf, X, Y - 0.5), bilinear(vf, X - 0.5, Y)


def fire_wind_sample(u3, v3, phi, hgt, z0, i, j, sr_x, sr_y, zf=6.1, g=G):
    """(u, v) at fire cell (i, j), evaluating only the staggered points it
    needs (for sampled checks on large meshes)."""
    u3 = np.asarray(u3)
    v3 = np.asarray(v3)
    z0 = np.asarray(z0, dtype=np.float64)
    phi = np.asarray(phi)
    hgt = np.asarray(hgt)
    nay, nax = hgt.shape
    cols = {}

    def zc_col(J, I):
        if (J, I) not in cols:
            cols[(J, I)] = (0.5 * (phi[:-1, J, I].astype(np.float64)
                                   + phi[1:, J, I].astype(np.float64)) / g - float(hgt[J, I]))
        return cols[(J, I)]

    class ZC:   # zc[:, J, I] on demand
        shape = (phi.shape[0] - 1, nay, nax)

        def __getitem__(self, key):
            _, J, I = key
            return zc_col(J, I)

    zc = ZC()
    X = (i + 0.5) / sr_x
    Y = (j + 0.5) / sr_y
    u = bilinear_fn(lambda J, I: u_point(u3, zc, z0, I, J, zf), nax + 1, nay, X, Y - 0.5)
    v = bilinear_fn(lambda J, I: v_point(v3, zc, z0, I, J, zf), nax, nay + 1, X - 0.5, Y)
    return u, v


def fire_wind(u3, v3, phi, hgt, z0, nx, ny, sr_x, sr_y, zf=6.1, g=G):
    """(u, v) on the fire mesh [ny][nx] (pure Python loops: small cases)."""
    uf, vf = staggered_surface_wind(u3, v3, phi, hgt, z0, zf, g)
    u = np.zeros((ny, nx))
    v = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            u[j, i], v[j, i] = fire_wind_at(uf, vf, i, j, sr_x, sr_y)
    return u, v
