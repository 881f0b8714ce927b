"""Python binding of the HIP fire-step library (``libfire_gfx950.so``).

Argument marshalling only: torch tensors provide device memory and the
stream; every step of the method runs in the library's HIP kernels.  The
names follow the C ABI in ``include/fire.h``.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfire_gfx950.so")

FIRE_F32, FIRE_F64 = 0, 1
STATUS_BOUNDARY, STATUS_NONFINITE = 1, 2
ERR_BOUNDARY = -4
ERR_NONFINITE = -5
ERR_TOO_LARGE = -7
WIND_STATIC_BYTES = 16 << 20
ENS_GRID = 0          # fire_ens_set_schedule: one work-group per tile
ENS_RESIDENT = 1      # resident work-groups over per-band tile counters
MAX_IGNITIONS = 8
NCOEF = 10
COEF_NAMES = ("S0", "R0", "b", "c", "d", "e", "m", "Tf", "Ch", "Cq")


class FireError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class fire_mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("sr_x", C.c_int32), ("sr_y", C.c_int32), ("dtype", C.c_int32),
                ("reserved", C.c_int32)]


class fire_fuel(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "windrf", "tf", "weight", "fgi", "fueldepthm", "savr", "fuelmce", "fueldens", "st",
        "se", "cmbcnst", "fuelmc_g", "ros_mult")] + [("ichap", C.c_int32), ("reserved", C.c_int32)]


class fire_ignition(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "ax", "ay", "bx", "by", "t_start", "radius", "ros", "vx", "vy", "t_end")]


class fire_params(C.Structure):
    _fields_ = [("viscosity", C.c_double), ("psi_init", C.c_double), ("wind_cap", C.c_double),
                ("ros_cap", C.c_double), ("t0", C.c_double), ("guard_width", C.c_int32),
                ("boundary_policy", C.c_int32), ("viscosity_mode", C.c_int32),
                ("reserved", C.c_int32)]


class fire_wind_grid(C.Structure):
    _fields_ = [("nax", C.c_int32), ("nay", C.c_int32), ("nz", C.c_int32), ("sr_x", C.c_int32),
                ("sr_y", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("dtype", C.c_int32),
                ("zf", C.c_double), ("g", C.c_double)]


class fire_view(C.Structure):
    _fields_ = [("psi", C.c_void_p), ("tign", C.c_void_p), ("frac", C.c_void_p),
                ("t", C.c_double)]


_lib = None


def lib():
    """Load the library; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP fire library not built: {LIB_PATH} missing "
                               "(run paper_1102_1343_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.fire_state_bytes.argtypes = [P(fire_mesh), C.c_int32]
        L.fire_state_bytes.restype = C.c_size_t
        L.fire_init.argtypes = [P(vp), P(fire_mesh), P(fire_fuel), C.c_int32, vp, vp, vp,
                                P(fire_ignition), C.c_int32, P(fire_params), vp, C.c_size_t, vp]
        L.fire_step.argtypes = [vp, vp, vp, C.c_double, vp, vp, P(fire_view)]
        L.fire_get_state.argtypes = [vp, P(fire_view)]
        L.fire_set_state.argtypes = [vp, vp, vp, vp, C.c_double]
        L.fire_status.argtypes = [vp]
        L.fire_coef.argtypes = [vp, P(C.c_double), C.c_int32]
        L.fire_ros_eval.argtypes = [vp, vp, vp, vp, vp, C.c_int64]
        L.fire_set_tile.argtypes = [vp, C.c_int32, C.c_int32]
        L.fire_get_tile.argtypes = [vp, P(C.c_int32), P(C.c_int32)]
        L.fire_set_stream.argtypes = [vp, vp]
        L.fire_default_tile.argtypes = [P(fire_mesh), P(C.c_int32), P(C.c_int32)]
        L.fire_strerror.argtypes = [C.c_int]
        L.fire_strerror.restype = C.c_char_p
        L.fire_destroy.argtypes = [vp]
        L.fire_destroy.restype = None
        i64p, i32p = P(C.c_int64), P(C.c_int32)
        L.fire_ens_layout.argtypes = [P(fire_mesh), C.c_int32, i64p, i64p]
        L.fire_ens_state_bytes.argtypes = [P(fire_mesh), C.c_int32, C.c_int32]
        L.fire_ens_state_bytes.restype = C.c_size_t
        L.fire_ens_init.argtypes = [P(vp), P(fire_mesh), C.c_int32, P(fire_fuel), C.c_int32, vp,
                                    vp, vp, P(fire_ignition), i32p, P(fire_params), vp,
                                    C.c_size_t, vp]
        L.fire_ens_step.argtypes = [vp, vp, vp, C.c_double, vp, vp]
        L.fire_ens_get_state.argtypes = [vp, P(fire_view)]
        L.fire_ens_status.argtypes = [vp, i32p]
        L.fire_ens_set_tile.argtypes = [vp, C.c_int32, C.c_int32]
        L.fire_ens_get_tile.argtypes = [vp, i32p, i32p]
        L.fire_ens_set_schedule.argtypes = [vp, C.c_int32]
        L.fire_ens_get_schedule.argtypes = [vp, i32p]
        L.fire_ens_tune_bytes.argtypes = [vp]
        L.fire_ens_tune_bytes.restype = C.c_size_t
        L.fire_ens_autotune.argtypes = [vp, vp, vp, C.c_double, vp, vp, i32p, C.c_int32,
                                        C.c_int32, vp, C.c_size_t, i32p]
        L.fire_ens_set_stream.argtypes = [vp, vp]
        L.fire_ens_destroy.argtypes = [vp]
        L.fire_ens_destroy.restype = None
        L.fire_adj_bytes.argtypes = [P(fire_mesh), C.c_int32, C.c_int32, C.c_int32]
        L.fire_adj_bytes.restype = C.c_size_t
        L.fire_adj_init.argtypes = [P(vp), vp, C.c_int32, C.c_int32, vp, C.c_size_t]
        L.fire_adj_forward.argtypes = [vp, vp, vp, C.c_double]
        L.fire_adj_backward.argtypes = [vp, vp, vp, vp, P(C.c_double), P(C.c_double)]
        L.fire_adj_destroy.argtypes = [vp]
        L.fire_adj_destroy.restype = None
        L.fire_wind_scratch_bytes.argtypes = [P(fire_wind_grid)]
        L.fire_wind_scratch_bytes.restype = C.c_size_t
        L.fire_wind_interp.argtypes = [P(fire_wind_grid), vp, vp, vp, vp, vp, vp, vp, vp,
                                       C.c_size_t, vp]
        L.fire_wind_interp_static.argtypes = [P(fire_wind_grid), vp, vp, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def default_tile(nx, ny, dx, dy, sr_x, sr_y, dtype=torch.float32):
    """The tile shape a context for this mesh starts with (fire_default_tile;
    host only)."""
    m = fire_mesh(int(nx), int(ny), float(dx), float(dy), int(sr_x), int(sr_y),
                  FIRE_F64 if dtype == torch.float64 else FIRE_F32, 0)
    a, b = C.c_int32(), C.c_int32()
    _check(lib().fire_default_tile(C.byref(m), C.byref(a), C.byref(b)), "fire_default_tile")
    return a.value, b.value


def strerror(code: int) -> str:
    return lib().fire_strerror(int(code)).decode()


def _check(code, what):
    if code != 0:
        raise FireError(code, what)


def _fuel_array(fuels):
    arr = (fire_fuel * len(fuels))()
    for k, f in enumerate(fuels):
        for name, typ in fire_fuel._fields_:
            if name != "reserved":
                setattr(arr[k], name, typ(f[name]))
    return arr


def _ign_array(igns):
    arr = (fire_ignition * max(1, len(igns)))()
    for k, g in enumerate(igns):
        for name, _ in fire_ignition._fields_:
            setattr(arr[k], name, float(g[name]))
    return arr


def _need(t, name, shape=None, dtype=None, device=None, numel=None):
    """Raise ValueError unless ``t`` is a contiguous CUDA tensor on ``device``
    with the given dtype and shape (or element count).  Runs before any
    pointer reaches the library, which has no way to check them."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: expected a CUDA tensor, got one on {t.device}")
    if device is not None and t.device != torch.device(device):
        raise ValueError(f"{name}: expected a tensor on {device}, got one on {t.device}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return t


def _cuda_device(device):
    d = torch.device(device)
    if d.type != "cuda":
        raise ValueError(f"the fire library runs on a GPU; device {d} is not a CUDA device")
    return torch.device("cuda", torch.cuda.current_device() if d.index is None else d.index)


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Fire:
    """One fire domain on one GPU, driven through the C ABI.

    ``fuels`` are dicts with the ``fire_fuel`` field names, ``cat`` a uint8
    [ny, nx] category map, ``dzdx``/``dzdy`` the terrain gradient,
    ``ignitions`` dicts with the ``fire_ignition`` field names.  Host arrays
    are copied to the device once; device tensors are used in place.
    """

    def __init__(self, nx, ny, dx, dy, sr_x, sr_y, fuels, cat, dzdx, dzdy, ignitions=(),
                 dtype=torch.float32, device="cuda", viscosity=0.4, psi_init=0.0, wind_cap=30.0,
                 ros_cap=math.inf, t0=0.0, guard_width=1, boundary_policy=0, viscosity_mode=0,
                 stream=None):
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        if len(ignitions) > MAX_IGNITIONS:
            raise ValueError(f"at most {MAX_IGNITIONS} ignitions")
        self.dtype = dtype
        self.device = _cuda_device(device)
        self.nx, self.ny = int(nx), int(ny)
        self.nax = -(-self.nx // int(sr_x))
        self.nay = -(-self.ny // int(sr_y))
        self.mesh = fire_mesh(self.nx, self.ny, float(dx), float(dy), int(sr_x), int(sr_y),
                              FIRE_F64 if dtype == torch.float64 else FIRE_F32, 0)
        self.ncat = len(fuels)
        self.nign = len(ignitions)
        self.cat = self._dev(cat, torch.uint8)
        if int(self.cat.max()) >= self.ncat:
            raise ValueError("fuel category map holds a value >= number of fuels")
        self.dzdx = self._dev(dzdx, dtype)
        self.dzdy = self._dev(dzdy, dtype)
        self.params = fire_params(float(viscosity), float(psi_init), float(wind_cap),
                                  float(ros_cap), float(t0), int(guard_width),
                                  int(boundary_policy), int(viscosity_mode), 0)
        nbytes = lib().fire_state_bytes(C.byref(self.mesh), self.ncat)
        if nbytes == 0:
            raise FireError(-1, "fire_state_bytes")
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        pad = (-self.arena.data_ptr()) % 256
        self._base = self.arena.data_ptr() + pad
        self._stream = stream
        fuels_c = _fuel_array(fuels)
        ign_c = _ign_array(list(ignitions))
        ctx = C.c_void_p()
        _check(lib().fire_init(C.byref(ctx), C.byref(self.mesh), fuels_c, self.ncat,
                               C.c_void_p(self.cat.data_ptr()), C.c_void_p(self.dzdx.data_ptr()),
                               C.c_void_p(self.dzdy.data_ptr()), ign_c, len(ignitions),
                               C.byref(self.params), C.c_void_p(self._base), nbytes,
                               _stream_handle(stream)), "fire_init")
        self._ctx = ctx
        self._pad = pad

    @classmethod
    def from_problem(cls, prob, dtype=torch.float32, device="cuda", **kw):
        """Build from a ``synth.Problem`` (same inputs the oracle takes)."""
        p = dict(prob.params)
        p.update(kw)
        return cls(prob.nx, prob.ny, prob.dx, prob.dy, prob.sr_x, prob.sr_y, prob.fuels,
                   prob.cat, prob.dzdx, prob.dzdy, prob.ignitions, dtype=dtype, device=device,
                   **{k: v for k, v in p.items() if k in (
                       "viscosity", "psi_init", "wind_cap", "ros_cap", "t0", "guard_width",
                       "boundary_policy", "viscosity_mode", "stream")})

    def _dev(self, a, dtype):
        if isinstance(a, torch.Tensor):
            t = a.to(device=self.device, dtype=dtype)
        else:
            t = torch.from_numpy(np.ascontiguousarray(a)).to(device=self.device, dtype=dtype)
        t = t.contiguous()
        if tuple(t.shape) != (self.ny, self.nx):
            raise ValueError(f"expected shape {(self.ny, self.nx)}, got {tuple(t.shape)}")
        return t

    # ------------------------------------------------------------ calls
    def new_flux(self):
        z = lambda: torch.empty((self.nay, self.nax), dtype=self.dtype, device=self.device)
        return z(), z()

    def step(self, u, v, dt, flux_sens=None, flux_lat=None, check=True):
        """One fire step; returns (flux_sens, flux_lat) on the atmosphere mesh.
        Raises FireError on an error code (FIRE_ERR_BOUNDARY under the stop
        policy) unless ``check`` is False, in which case the code is returned
        as the third element."""
        if flux_sens is None or flux_lat is None:
            flux_sens, flux_lat = self.new_flux()
        grid = (self.ny, self.nx)
        _need(u, "u", grid, self.dtype, self.device)
        _need(v, "v", grid, self.dtype, self.device)
        atm = (self.nay, self.nax)
        _need(flux_sens, "flux_sens", atm, self.dtype, self.device)
        _need(flux_lat, "flux_lat", atm, self.dtype, self.device)
        rc = lib().fire_step(self._ctx, C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()),
                             float(dt), C.c_void_p(flux_sens.data_ptr()),
                             C.c_void_p(flux_lat.data_ptr()), None)
        if check:
            _check(rc, "fire_step")
            return flux_sens, flux_lat
        return flux_sens, flux_lat, rc

    def _view(self):
        vw = fire_view()
        _check(lib().fire_get_state(self._ctx, C.byref(vw)), "fire_get_state")
        return vw

    def _slice(self, ptr):
        off = ptr - self.arena.data_ptr()
        es = 8 if self.dtype == torch.float64 else 4
        n = self.nx * self.ny
        return self.arena[off:off + n * es].view(self.dtype).view(self.ny, self.nx)

    @property
    def psi(self):
        return self._slice(self._view().psi)

    @property
    def tign(self):
        return self._slice(self._view().tign)

    @property
    def frac(self):
        return self._slice(self._view().frac)

    @property
    def t(self):
        return self._view().t

    def set_state(self, psi, tign, frac, t):
        psi, tign, frac = (self._dev(a, self.dtype) for a in (psi, tign, frac))
        _check(lib().fire_set_state(self._ctx, C.c_void_p(psi.data_ptr()),
                                    C.c_void_p(tign.data_ptr()), C.c_void_p(frac.data_ptr()),
                                    float(t)), "fire_set_state")
        (self._stream or torch.cuda.current_stream()).synchronize()

    def status(self) -> int:
        rc = lib().fire_status(self._ctx)
        if rc < 0:
            raise FireError(rc, "fire_status")
        return rc

    def coef(self) -> np.ndarray:
        out = np.zeros((self.ncat, NCOEF))
        _check(lib().fire_coef(self._ctx, out.ctypes.data_as(C.POINTER(C.c_double)), self.ncat),
               "fire_coef")
        return out

    def ros_eval(self, cat, un, tn):
        n = un.numel() if isinstance(un, torch.Tensor) else -1
        _need(un, "un", dtype=self.dtype, device=self.device)
        _need(tn, "tn", dtype=self.dtype, device=self.device, numel=n)
        _need(cat, "cat", dtype=torch.uint8, device=self.device, numel=n)
        S = torch.empty_like(un)
        _check(lib().fire_ros_eval(self._ctx, C.c_void_p(cat.data_ptr()),
                                   C.c_void_p(un.data_ptr()), C.c_void_p(tn.data_ptr()),
                                   C.c_void_p(S.data_ptr()), un.numel()), "fire_ros_eval")
        return S

    def set_tile(self, tile_x, tile_y):
        _check(lib().fire_set_tile(self._ctx, int(tile_x), int(tile_y)), "fire_set_tile")

    def set_stream(self, stream):
        """Enqueue later calls on ``stream`` (a torch.cuda.Stream)."""
        self._stream = stream
        _check(lib().fire_set_stream(self._ctx, _stream_handle(stream)), "fire_set_stream")

    def get_tile(self):
        a, b = C.c_int32(), C.c_int32()
        _check(lib().fire_get_tile(self._ctx, C.byref(a), C.byref(b)), "fire_get_tile")
        return a.value, b.value

    def close(self):
        if getattr(self, "_ctx", None):
            lib().fire_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FireEnsemble:
    """Many fire domains of different sizes stepped by one launch per step.

    ``members`` are ``synth.Problem``-like objects (nx, ny, dx, dy, sr_x,
    sr_y, cat, dzdx, dzdy, ignitions); all share ``fuels`` and the
    parameters.  Per-cell arrays are concatenated 1-D tensors: member k owns
    elements ``cell_off[k]:cell_off[k+1]`` (row-major [ny_k, nx_k]);
    atmosphere arrays likewise with ``atm_off``.
    """

    def __init__(self, members, fuels, dtype=torch.float32, device="cuda", viscosity=0.4,
                 psi_init=0.0, wind_cap=30.0, ros_cap=math.inf, t0=0.0, guard_width=1,
                 viscosity_mode=0, stream=None):
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.dtype = dtype
        self.device = _cuda_device(device)
        self.ndom = len(members)
        fd = FIRE_F64 if dtype == torch.float64 else FIRE_F32
        self.meshes = (fire_mesh * self.ndom)()
        for k, m in enumerate(members):
            self.meshes[k] = fire_mesh(int(m.nx), int(m.ny), float(m.dx), float(m.dy),
                                       int(m.sr_x), int(m.sr_y), fd, 0)
        self.shapes = [(int(m.ny), int(m.nx)) for m in members]
        self.atm_shapes = [(-(-int(m.ny) // int(m.sr_y)), -(-int(m.nx) // int(m.sr_x)))
                           for m in members]
        co = (C.c_int64 * (self.ndom + 1))()
        ao = (C.c_int64 * (self.ndom + 1))()
        _check(lib().fire_ens_layout(self.meshes, self.ndom, co, ao), "fire_ens_layout")
        self.cell_off = np.array(co[:], dtype=np.int64)
        self.atm_off = np.array(ao[:], dtype=np.int64)
        self.ncat = len(fuels)
        self.cat = self.concat([m.cat for m in members], torch.uint8)
        if int(self.cat.max()) >= self.ncat:
            raise ValueError("fuel category map holds a value >= number of fuels")
        self.dzdx = self.concat([m.dzdx for m in members])
        self.dzdy = self.concat([m.dzdy for m in members])
        igs, nign = [], (C.c_int32 * self.ndom)()
        for k, m in enumerate(members):
            if len(m.ignitions) > MAX_IGNITIONS:
                raise ValueError(f"member {k}: at most {MAX_IGNITIONS} ignitions")
            igs += list(m.ignitions)
            nign[k] = len(m.ignitions)
        ign_c = _ign_array(igs)
        self.params = fire_params(float(viscosity), float(psi_init), float(wind_cap),
                                  float(ros_cap), float(t0), int(guard_width), 1,
                                  int(viscosity_mode), 0)
        nbytes = lib().fire_ens_state_bytes(self.meshes, self.ndom, self.ncat)
        if nbytes == 0:
            raise FireError(-1, "fire_ens_state_bytes")
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._base = self.arena.data_ptr() + (-self.arena.data_ptr()) % 256
        self._stream = stream
        h = C.c_void_p()
        _check(lib().fire_ens_init(C.byref(h), self.meshes, self.ndom, _fuel_array(fuels),
                                   self.ncat, C.c_void_p(self.cat.data_ptr()),
                                   C.c_void_p(self.dzdx.data_ptr()),
                                   C.c_void_p(self.dzdy.data_ptr()), ign_c, nign,
                                   C.byref(self.params), C.c_void_p(self._base), nbytes,
                                   _stream_handle(stream)), "fire_ens_init")
        self._h = h

    @classmethod
    def from_problems(cls, probs, dtype=torch.float32, device="cuda", **kw):
        p = dict(probs[0].params)
        p.update(kw)
        return cls(probs, probs[0].fuels, dtype=dtype, device=device,
                   **{k: v for k, v in p.items() if k in (
                       "viscosity", "psi_init", "wind_cap", "ros_cap", "t0", "guard_width",
                       "viscosity_mode", "stream")})

    @property
    def ncells(self):
        return int(self.cell_off[-1])

    def concat(self, arrays, dtype=None):
        """Concatenate per-member [ny_k, nx_k] arrays into one device tensor."""
        dtype = dtype or self.dtype
        parts = []
        for k, a in enumerate(arrays):
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            if tuple(t.shape) != self.shapes[k]:
                raise ValueError(f"member {k}: expected shape {self.shapes[k]}, "
                                 f"got {tuple(t.shape)}")
            parts.append(t.reshape(-1).to(device=self.device, dtype=dtype))
        return torch.cat(parts).contiguous()

    def member(self, flat, k, atm=False):
        """View of member k's block of a concatenated array."""
        off, shp = (self.atm_off, self.atm_shapes) if atm else (self.cell_off, self.shapes)
        return flat[int(off[k]):int(off[k + 1])].view(shp[k])

    def new_flux(self):
        n = int(self.atm_off[-1])
        z = lambda: torch.empty(n, dtype=self.dtype, device=self.device)
        return z(), z()

    def step(self, u, v, dt, flux_sens=None, flux_lat=None):
        if flux_sens is None or flux_lat is None:
            flux_sens, flux_lat = self.new_flux()
        self._check_wind(u, v)
        natm = int(self.atm_off[-1])
        _need(flux_sens, "flux_sens", dtype=self.dtype, device=self.device, numel=natm)
        _need(flux_lat, "flux_lat", dtype=self.dtype, device=self.device, numel=natm)
        _check(lib().fire_ens_step(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()),
                                   float(dt), C.c_void_p(flux_sens.data_ptr()),
                                   C.c_void_p(flux_lat.data_ptr())), "fire_ens_step")
        return flux_sens, flux_lat

    def _check_wind(self, u, v):
        _need(u, "u", dtype=self.dtype, device=self.device, numel=self.ncells)
        _need(v, "v", dtype=self.dtype, device=self.device, numel=self.ncells)

    def _view(self):
        vw = fire_view()
        _check(lib().fire_ens_get_state(self._h, C.byref(vw)), "fire_ens_get_state")
        return vw

    def _slice(self, ptr):
        off = ptr - self.arena.data_ptr()
        es = 8 if self.dtype == torch.float64 else 4
        return self.arena[off:off + self.ncells * es].view(self.dtype)

    @property
    def psi(self):
        return self._slice(self._view().psi)

    @property
    def tign(self):
        return self._slice(self._view().tign)

    @property
    def frac(self):
        return self._slice(self._view().frac)

    @property
    def t(self):
        return self._view().t

    def status(self) -> np.ndarray:
        out = (C.c_int32 * self.ndom)()
        _check(lib().fire_ens_status(self._h, out), "fire_ens_status")
        return np.array(out[:], dtype=np.int32)

    def set_tile(self, tile_x, tile_y):
        _check(lib().fire_ens_set_tile(self._h, int(tile_x), int(tile_y)), "fire_ens_set_tile")

    def set_stream(self, stream):
        """Enqueue later calls on ``stream`` (a torch.cuda.Stream)."""
        self._stream = stream
        _check(lib().fire_ens_set_stream(self._h, _stream_handle(stream)), "fire_ens_set_stream")

    def get_tile(self):
        a, b = C.c_int32(), C.c_int32()
        _check(lib().fire_ens_get_tile(self._h, C.byref(a), C.byref(b)), "fire_ens_get_tile")
        return a.value, b.value

    def set_schedule(self, resident: bool):
        """One work-group per tile (False, the default) or resident
        work-groups taking tiles from per-band counters (True)."""
        _check(lib().fire_ens_set_schedule(self._h, ENS_RESIDENT if resident else ENS_GRID),
               "fire_ens_set_schedule")

    def get_schedule(self) -> bool:
        a = C.c_int32()
        _check(lib().fire_ens_get_schedule(self._h, C.byref(a)), "fire_ens_get_schedule")
        return a.value == ENS_RESIDENT

    def autotune(self, u, v, dt, candidates, reps=5):
        """Time each (tile_x, tile_y) candidate, keep the fastest; the state is
        left as it was.  Returns the chosen shape."""
        self._check_wind(u, v)
        nb = lib().fire_ens_tune_bytes(self._h)
        scratch = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        base = scratch.data_ptr() + (-scratch.data_ptr()) % 256
        cand = (C.c_int32 * (2 * len(candidates)))(*[int(x) for c in candidates for x in c])
        best = (C.c_int32 * 2)()
        fs, fl = self.new_flux()
        _check(lib().fire_ens_autotune(self._h, C.c_void_p(u.data_ptr()),
                                       C.c_void_p(v.data_ptr()), float(dt),
                                       C.c_void_p(fs.data_ptr()), C.c_void_p(fl.data_ptr()),
                                       cand, len(candidates), int(reps), C.c_void_p(base), nb,
                                       best), "fire_ens_autotune")
        return best[0], best[1]

    def close(self):
        if getattr(self, "_h", None):
            lib().fire_ens_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FireAdjoint:
    """Differentiable run of a ``Fire`` context: ``forward`` steps it
    ``nsteps`` times under one wind, keeping psi every ``every`` steps;
    ``backward(dF)`` returns dL/du, dL/dv (device tensors), dL/dm_k (numpy,
    per category) and dL/d(shift) (numpy [nign, 2]) for dF = dL/dF_end."""

    def __init__(self, fire, nsteps, every=50):
        self.fire = fire
        self.nsteps, self.every = int(nsteps), int(every)
        nb = lib().fire_adj_bytes(C.byref(fire.mesh), fire.ncat, self.nsteps, self.every)
        if nb == 0:
            raise FireError(-1, "fire_adj_bytes")
        self.scratch = torch.empty(nb + 256, dtype=torch.uint8, device=fire.device)
        base = self.scratch.data_ptr() + (-self.scratch.data_ptr()) % 256
        h = C.c_void_p()
        _check(lib().fire_adj_init(C.byref(h), fire._ctx, self.nsteps, self.every,
                                   C.c_void_p(base), nb), "fire_adj_init")
        self._h = h
        self._wind = None

    def forward(self, u, v, dt):
        f = self.fire
        _need(u, "u", (f.ny, f.nx), f.dtype, f.device)
        _need(v, "v", (f.ny, f.nx), f.dtype, f.device)
        self._wind = (u, v)     # the library keeps the pointers until backward
        _check(lib().fire_adj_forward(self._h, C.c_void_p(u.data_ptr()),
                                      C.c_void_p(v.data_ptr()), float(dt)), "fire_adj_forward")
        return f.frac

    def backward(self, dF):
        f = self.fire
        _need(dF, "dF", (f.ny, f.nx), f.dtype, f.device)
        gu = torch.empty_like(dF)
        gv = torch.empty_like(dF)
        gm = np.zeros(f.ncat)
        gs = np.zeros((max(1, f.nign), 2))
        _check(lib().fire_adj_backward(self._h, C.c_void_p(dF.data_ptr()),
                                       C.c_void_p(gu.data_ptr()), C.c_void_p(gv.data_ptr()),
                                       gm.ctypes.data_as(C.POINTER(C.c_double)),
                                       gs.ctypes.data_as(C.POINTER(C.c_double))),
               "fire_adj_backward")
        return gu, gv, gm, gs[:f.nign]

    def close(self):
        if getattr(self, "_h", None):
            lib().fire_adj_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shifted_ignitions(ignitions, shift):
    """Ignitions translated by shift[g] = (dx, dy) metres (start and end)."""
    out = []
    for g, (sx, sy) in zip(ignitions, shift):
        out.append(dict(g, ax=g["ax"] + sx, ay=g["ay"] + sy, bx=g["bx"] + sx, by=g["by"] + sy))
    return out


class FireRun(torch.autograd.Function):
    """F_end = run(u, v, m, shift): ``nsteps`` fire steps of ``prob`` (a
    ``synth.Problem``) under the wind (u, v), with per-category spread
    multipliers m and ignitions translated by shift [nign, 2]; differentiable
    in all four through the hand-written adjoint."""

    @staticmethod
    def forward(ctx, u, v, mult, shift, prob, nsteps, every=50, dtype=torch.float64):
        for name, t in (("u", u), ("v", v)):
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
                raise ValueError(f"{name}: FireRun needs CUDA tensors (the run is on the GPU)")
        fuels = [dict(f, ros_mult=float(m)) for f, m in zip(prob.fuels, mult.tolist())]
        igns = shifted_ignitions(prob.ignitions, shift.detach().cpu().tolist())
        p = dict(prob.params)
        fire = Fire(prob.nx, prob.ny, prob.dx, prob.dy, prob.sr_x, prob.sr_y, fuels, prob.cat,
                    prob.dzdx, prob.dzdy, igns, dtype=dtype, device=u.device,
                    **{k: v_ for k, v_ in p.items() if k in (
                        "viscosity", "psi_init", "wind_cap", "ros_cap", "t0", "guard_width",
                        "boundary_policy", "viscosity_mode")})
        adj = FireAdjoint(fire, nsteps, every)
        uu = u.detach().to(dtype).contiguous()
        vv = v.detach().to(dtype).contiguous()
        F = adj.forward(uu, vv, prob.dt).clone()
        ctx.adj = adj
        ctx.keep = (fire, uu, vv)
        ctx.meta = (u.dtype, v.dtype, mult.dtype, mult.device, shift.dtype, shift.device)
        return F

    @staticmethod
    def backward(ctx, gF):
        udt, vdt, mdt, mdev, sdt, sdev = ctx.meta
        fire = ctx.keep[0]
        gu, gv, gm, gs = ctx.adj.backward(gF.detach().to(fire.dtype).contiguous())
        return (gu.to(udt), gv.to(vdt), torch.from_numpy(gm).to(mdev, mdt),
                torch.from_numpy(np.ascontiguousarray(gs)).to(sdev, sdt), None, None, None, None)


def wind_interp(u3, v3, phi, hgt, z0, nx, ny, sr_x, sr_y, zf=6.1, g=9.81, stream=None,
                out=None, scratch=None):
    """Surface wind on the fire mesh [ny, nx] from the atmosphere's staggered
    u3 [nz, nay, nax+1], v3 [nz, nay+1, nax], geopotential phi
    [nz+1, nay, nax], terrain height and roughness [nay, nax] (device
    tensors of one floating dtype).  Returns (u, v) device tensors (``out``
    if given).  With a caller-kept ``scratch`` (uint8 device tensor of at
    least wind_scratch_bytes() + 256) the call does not wait."""
    _need(u3, "u3")
    dt, dev = u3.dtype, u3.device
    if dt not in (torch.float32, torch.float64):
        raise ValueError("float32 or float64 tensors expected")
    if u3.dim() != 3:
        raise ValueError("u3: expected [nz, nay, nax + 1]")
    nz, nay, nax1 = u3.shape
    nax = nax1 - 1
    shapes = {"v3": (v3, (nz, nay + 1, nax)), "phi": (phi, (nz + 1, nay, nax)),
              "hgt": (hgt, (nay, nax)), "z0": (z0, (nay, nax))}
    for name, (t, shp) in shapes.items():
        _need(t, name, shp, dt, dev)
    grid = fire_wind_grid(nax, nay, nz, int(sr_x), int(sr_y), int(nx), int(ny),
                          FIRE_F64 if dt == torch.float64 else FIRE_F32, float(zf), float(g))
    nb = lib().fire_wind_scratch_bytes(C.byref(grid))
    if nb == 0:
        raise FireError(-1, "fire_wind_scratch_bytes")
    own = scratch is None
    if own:
        scratch = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
    else:
        _need(scratch, "scratch", dtype=torch.uint8, device=dev)
        if scratch.numel() < nb + 256:
            raise ValueError("scratch too small")
    base = scratch.data_ptr() + (-scratch.data_ptr()) % 256
    if out is None:
        u = torch.empty((int(ny), int(nx)), dtype=dt, device=dev)
        v = torch.empty_like(u)
    else:
        u, v = out
        _need(u, "out[0]", (int(ny), int(nx)), dt, dev)
        _need(v, "out[1]", (int(ny), int(nx)), dt, dev)
    _check(lib().fire_wind_interp(C.byref(grid), C.c_void_p(u3.data_ptr()),
                                  C.c_void_p(v3.data_ptr()), C.c_void_p(phi.data_ptr()),
                                  C.c_void_p(hgt.data_ptr()), C.c_void_p(z0.data_ptr()),
                                  C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()),
                                  C.c_void_p(base), nb, _stream_handle(stream)),
           "fire_wind_interp")
    if own:   # the scratch must outlive the asynchronous kernels
        (stream or torch.cuda.current_stream()).synchronize()
    return u, v


def wind_interp_static(u3, v3, phi, hgt, z0, nx, ny, sr_x, sr_y, out, zf=6.1, g=9.81,
                       stream=None):
    """wind_interp through fire_wind_interp_static: the library's own fixed
    scratch, nothing allocated; ``out`` = (u, v) [ny, nx] device tensors are
    required.  Overlapping calls on one GPU race (they share the scratch)."""
    _need(u3, "u3")
    dt, dev = u3.dtype, u3.device
    if dt not in (torch.float32, torch.float64) or u3.dim() != 3:
        raise ValueError("u3: expected a float32 or float64 [nz, nay, nax + 1] tensor")
    nz, nay, nax1 = u3.shape
    nax = nax1 - 1
    for name, t, shp in (("v3", v3, (nz, nay + 1, nax)), ("phi", phi, (nz + 1, nay, nax)),
                         ("hgt", hgt, (nay, nax)), ("z0", z0, (nay, nax))):
        _need(t, name, shp, dt, dev)
    u, v = out
    _need(u, "out[0]", (int(ny), int(nx)), dt, dev)
    _need(v, "out[1]", (int(ny), int(nx)), dt, dev)
    grid = fire_wind_grid(nax, nay, nz, int(sr_x), int(sr_y), int(nx), int(ny),
                          FIRE_F64 if dt == torch.float64 else FIRE_F32, float(zf), float(g))
    _check(lib().fire_wind_interp_static(C.byref(grid), C.c_void_p(u3.data_ptr()),
                                         C.c_void_p(v3.data_ptr()), C.c_void_p(phi.data_ptr()),
                                         C.c_void_p(hgt.data_ptr()), C.c_void_p(z0.data_ptr()),
                                         C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()),
                                         _stream_handle(stream)), "fire_wind_interp_static")
    return u, v


def wind_scratch_bytes(nax, nay, nz, nx, ny, sr_x, sr_y, dtype=torch.float32):
    grid = fire_wind_grid(nax, nay, nz, sr_x, sr_y, nx, ny,
                          FIRE_F64 if dtype == torch.float64 else FIRE_F32, 6.1, 9.81)
    return lib().fire_wind_scratch_bytes(C.byref(grid))
