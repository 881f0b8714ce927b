"""FP64 CPU oracle of the WRF-Fire fire-mesh time step (arXiv:1102.1343).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package.  The product library never imports it.

The arithmetic lives in ``fire_oracle.c`` (plain C loops, double precision);
this module only builds that file with gcc and marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fire_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_fire.so")

BOUNDARY = 1
NONFINITE = 2

# coefficient table columns
S0, R0, B, CC, D, E, M, TF, CH, CQ = range(10)
NCOEF = 10

# intermediates of the Table 2 chain, in the order oracle_rothermel_terms
# writes them (English units: 1/ft, lb/ft^2, ft, lb/ft^3, BTU/lb, ft/min)
ROTHERMEL_TERMS = ("sigma", "w_l", "delta", "rho_P", "h", "w_0", "rho_b", "beta", "beta_op",
                   "A", "Gamma_max", "Gamma", "w_n", "eta_M", "eta_s", "I_R", "xi", "epsilon",
                   "Q_ig", "R0_ftmin", "R0_ms", "C", "B", "E", "U_a", "phi_W", "phi_S", "S_ms")


def build(force: bool = True) -> str:
    """Compile the oracle into ``liboracle_fire.so`` (gcc, -O3, OpenMP).
    Contraction into FMA is disabled so the result is the plain expression."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-std=c11", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Fuel(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "windrf", "tf", "weight", "fgi", "fueldepthm", "savr", "fuelmce", "fueldens",
        "st", "se", "cmbcnst", "fuelmc_g", "ros_mult")] + [("ichap", C.c_int32), ("pad_", C.c_int32)]


class _Ign(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "ax", "ay", "bx", "by", "t_start", "radius", "ros", "vx", "vy", "t_end")]


class _Mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("sr_x", C.c_int32), ("sr_y", C.c_int32)]


class _Prm(C.Structure):
    _fields_ = [("viscosity", C.c_double), ("viscosity_mode", C.c_int32),
                ("guard_width", C.c_int32), ("ros_cap", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.oracle_coef.argtypes = [C.POINTER(_Fuel), C.c_int, C.c_double, dp]
        L.oracle_ros_product.argtypes = [C.POINTER(_Fuel), C.c_double, C.c_double, C.c_double, dp]
        L.oracle_rothermel_terms.argtypes = [C.POINTER(_Fuel), C.c_double, C.c_double,
                                             C.c_double, dp]
        L.oracle_nterms.restype = C.c_int
        L.oracle_ros.argtypes = [dp, C.c_double, C.c_double, C.c_double]
        L.oracle_ros.restype = C.c_double
        L.oracle_extrapolate.argtypes = [dp, C.c_int, C.c_int, dp]
        L.oracle_godunov.argtypes = [C.c_double, C.c_double]
        L.oracle_godunov.restype = C.c_double
        L.oracle_subcell_beta.argtypes = [dp]
        L.oracle_subcell_beta.restype = C.c_double
        L.oracle_subcell_burned.argtypes = [dp, dp, C.c_double, C.c_double]
        L.oracle_subcell_burned.restype = C.c_double
        L.oracle_cell_frac.argtypes = [dp, dp, C.c_double, C.c_double]
        L.oracle_cell_frac.restype = C.c_double
        L.oracle_ign_active.argtypes = [C.POINTER(_Ign), C.c_double]
        L.oracle_ign_psi.argtypes = [C.POINTER(_Ign), C.c_double, C.c_double, C.c_double, dp]
        L.oracle_ign_psi.restype = C.c_double
        L.oracle_step.argtypes = [C.POINTER(_Mesh), dp, C.c_int, C.POINTER(C.c_uint8), dp, dp,
                                  dp, dp, C.POINTER(_Ign), C.c_int, C.POINTER(_Prm), C.c_double,
                                  C.c_double, dp, dp, dp, dp, dp, C.POINTER(C.c_int32)]
        L.oracle_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = None
        assert L.oracle_sizeof_fuel() == C.sizeof(_Fuel)
        assert L.oracle_sizeof_ign() == C.sizeof(_Ign)
        assert L.oracle_ncoef() == NCOEF
        assert L.oracle_nterms() == len(ROTHERMEL_TERMS)
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _fuels(fuels):
    arr = (_Fuel * len(fuels))()
    for k, f in enumerate(fuels):
        for name, _ in _Fuel._fields_:
            if name == "pad_":
                continue
            setattr(arr[k], name, type(getattr(arr[k], name))(f[name]))
    return arr


def _igns(igns):
    arr = (_Ign * max(1, len(igns)))()
    for k, g in enumerate(igns):
        for name, _ in _Ign._fields_:
            setattr(arr[k], name, float(g[name]))
    return arr


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    """Use ``n`` OpenMP threads in the oracle's loops from now on."""
    lib().oracle_set_threads(int(n))


# ---------------------------------------------------------------- pieces

def coef(fuels, wind_cap=30.0) -> np.ndarray:
    """Coefficient table [ncat, 10]: S0 R0 b c d e m T_f C_h C_q."""
    tab = np.zeros((len(fuels), NCOEF))
    rc = lib().oracle_coef(_fuels(fuels), len(fuels), wind_cap, _dptr(tab))
    if rc:
        raise ValueError("oracle_coef failed")
    return tab


def ros(row, U, tanphi, ros_cap=math.inf) -> float:
    row = np.ascontiguousarray(row, dtype=np.float64)
    return lib().oracle_ros(_dptr(row), float(U), float(tanphi), float(ros_cap))


def ros_product(f, U, tanphi, wind_cap=30.0) -> float:
    out = C.c_double()
    lib().oracle_ros_product(_fuels([f]), float(U), float(tanphi), float(wind_cap), C.byref(out))
    return out.value


def rothermel_terms(f, U, tanphi, wind_cap=30.0) -> dict:
    """Every intermediate of the Table 2 chain for fuel ``f`` (a non-chaparral
    fuel record) at the 6.1 m wind U (m/s) and slope tan(phi)."""
    out = np.zeros(len(ROTHERMEL_TERMS))
    rc = lib().oracle_rothermel_terms(_fuels([f]), float(U), float(tanphi), float(wind_cap),
                                      _dptr(out))
    if rc != len(ROTHERMEL_TERMS):
        raise ValueError("oracle_rothermel_terms failed (chaparral fuel?)")
    return dict(zip(ROTHERMEL_TERMS, out.tolist()))


def extrapolate(psi: np.ndarray) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    ny, nx = psi.shape
    ext = np.zeros((ny + 2, nx + 2))
    lib().oracle_extrapolate(_dptr(psi), nx, ny, _dptr(ext))
    return ext


def godunov(dm, dp) -> float:
    return lib().oracle_godunov(float(dm), float(dp))


def subcell_beta(psi4) -> float:
    return lib().oracle_subcell_beta(_dptr(np.ascontiguousarray(psi4, dtype=np.float64)))


def subcell_burned(psi4, ti4, t, Tf) -> float:
    return lib().oracle_subcell_burned(_dptr(np.ascontiguousarray(psi4, dtype=np.float64)),
                                       _dptr(np.ascontiguousarray(ti4, dtype=np.float64)),
                                       float(t), float(Tf))


def cell_frac(p9, t9, t, Tf) -> float:
    return lib().oracle_cell_frac(_dptr(np.ascontiguousarray(p9, dtype=np.float64).ravel()),
                                  _dptr(np.ascontiguousarray(t9, dtype=np.float64).ravel()),
                                  float(t), float(Tf))


def ign_active(g, t) -> bool:
    return bool(lib().oracle_ign_active(_igns([g]), float(t)))


def ign_psi(g, x, y, t):
    a = C.c_double()
    p = lib().oracle_ign_psi(_igns([g]), float(x), float(y), float(t), C.byref(a))
    return p, a.value


# ---------------------------------------------------------------- full run

class OracleFire:
    """Oracle fire model over a ``synth.Problem``-like description.

    State: ``psi``, ``tign``, ``frac`` ([ny, nx] float64), time ``t`` and the
    sticky ``status``.  ``step(u, v, dt)`` returns the sensible and latent flux
    on the atmosphere mesh.  Initial state (Sect. 4.4): psi = psi_init > 0
    (default: the domain diagonal, reading R17), no ignition time, F = 1.
    """

    def __init__(self, prob, viscosity=None, viscosity_mode=None, ros_cap=None, wind_cap=30.0,
                 guard_width=None, psi_init=0.0, t0=0.0):
        p = prob.params
        self.prob = prob
        self.nx, self.ny = prob.nx, prob.ny
        self.mesh = _Mesh(prob.nx, prob.ny, prob.dx, prob.dy, prob.sr_x, prob.sr_y)
        self.prm = _Prm(p.get("viscosity", 0.4) if viscosity is None else viscosity,
                        p.get("viscosity_mode", 0) if viscosity_mode is None else viscosity_mode,
                        p.get("guard_width", 1) if guard_width is None else guard_width,
                        p.get("ros_cap", math.inf) if ros_cap is None else ros_cap)
        self.tab = coef(prob.fuels, wind_cap)
        self.ncat = len(prob.fuels)
        self.cat = np.ascontiguousarray(prob.cat, dtype=np.uint8)
        self.gzx = np.ascontiguousarray(prob.dzdx, dtype=np.float64)
        self.gzy = np.ascontiguousarray(prob.dzdy, dtype=np.float64)
        self._ign = _igns(prob.ignitions)
        self.nign = len(prob.ignitions)
        if psi_init <= 0.0:
            psi_init = math.hypot(prob.nx * prob.dx, prob.ny * prob.dy)
        self.psi = np.full((prob.ny, prob.nx), float(psi_init))
        self.tign = np.full((prob.ny, prob.nx), math.inf)
        self.frac = np.ones((prob.ny, prob.nx))
        self.t = float(t0)
        self.status = 0
        self.nax = -(-prob.nx // prob.sr_x)
        self.nay = -(-prob.ny // prob.sr_y)

    def step(self, u, v, dt):
        u = np.ascontiguousarray(u, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        fs = np.zeros((self.nay, self.nax))
        fl = np.zeros((self.nay, self.nax))
        st = C.c_int32(0)
        rc = lib().oracle_step(C.byref(self.mesh), _dptr(self.tab), self.ncat,
                               self.cat.ctypes.data_as(C.POINTER(C.c_uint8)), _dptr(self.gzx),
                               _dptr(self.gzy), _dptr(u), _dptr(v), self._ign, self.nign,
                               C.byref(self.prm), self.t, float(dt), _dptr(self.psi),
                               _dptr(self.tign), _dptr(self.frac), _dptr(fs), _dptr(fl),
                               C.byref(st))
        if rc:
            raise ValueError(f"oracle_step failed ({rc})")
        self.status |= st.value
        self.t += float(dt)
        return fs, fl

    def run(self, steps=None, callback=None):
        prob = self.prob
        steps = prob.steps if steps is None else steps
        out = None
        for k in range(steps):
            u, v = prob.wind_at(k)
            out = self.step(u, v, prob.dt)
            if callback:
                callback(k, self, out)
        return out
