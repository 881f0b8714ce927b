"""The C ABI library loads on a machine without a GPU, exports every symbol
that include/fire.h declares, agrees with the header on struct layouts, and
rejects bad arguments before touching the device.  CPU only."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fire.h")
LIB = os.path.join(ROOT, "paper_1102_1343_amd", "libfire_gfx950.so")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fire_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts_match_header(tmp_path):
    from paper_1102_1343_amd import fire as F
    prog = tmp_path / "sz.c"
    prog.write_text('#include "fire.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(fire_mesh),'
                    'sizeof(fire_fuel), sizeof(fire_ignition), sizeof(fire_params),'
                    'sizeof(fire_view), offsetof(fire_params, guard_width));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(F.fire_mesh), C.sizeof(F.fire_fuel), C.sizeof(F.fire_ignition),
            C.sizeof(F.fire_params), C.sizeof(F.fire_view), F.fire_params.guard_width.offset]
    assert got == want


def test_state_bytes_and_errors_without_gpu(lib):
    from paper_1102_1343_amd import fire as F
    lib.fire_state_bytes.restype = C.c_size_t
    lib.fire_strerror.restype = C.c_char_p
    m = F.fire_mesh(128, 96, 6.0, 6.0, 10, 10, F.FIRE_F32, 0)
    n = 128 * 96
    nb = lib.fire_state_bytes(C.byref(m), 13)
    # psi x2, t_i, F (4 B each) plus the table, fuel staging, status word, the
    # step's ignition geometry (at most 1 KiB) and its per-tile set-up: a word
    # and 8 bounds for each of the 2 x 5 tiles of the default 120 x 20 tile,
    # 16 row offsets for each of ny + 48 rows (three 256-byte aligned parts)
    iset = 10 * (4 + 8 * 4) + 16 * (96 + 48) * 4
    assert 16 * n + iset <= nb <= 16 * n + 8 * 256 + 13 * (10 * 4 + 112) + 256 + 1024 + iset + 3 * 256
    m64 = F.fire_mesh(128, 96, 6.0, 6.0, 10, 10, F.FIRE_F64, 0)
    iset64 = 10 * (4 + 8 * 8) + 16 * (96 + 48) * 8
    nb64 = lib.fire_state_bytes(C.byref(m64), 13)
    assert 32 * n + iset64 <= nb64 <= 32 * n + 8 * 256 + 13 * (10 * 8 + 112) + 256 + 1024 + iset64 + 3 * 256
    # refinement 11: default tile 121 x 11, so 3 x 9 tiles of a 250 x 99 mesh
    m11 = F.fire_mesh(250, 99, 6.0, 6.0, 11, 11, F.FIRE_F32, 0)
    n11 = 250 * 99
    iset11 = 27 * (4 + 8 * 4) + 16 * (99 + 48) * 4
    nb11 = lib.fire_state_bytes(C.byref(m11), 13)
    assert 16 * n11 + iset11 <= nb11 <= 16 * n11 + 8 * 256 + 13 * (10 * 4 + 112) + 256 + 1024 + iset11 + 3 * 256
    for bad in (F.fire_mesh(1, 96, 6.0, 6.0, 10, 10, 0, 0), F.fire_mesh(128, 96, 0.0, 6.0, 10, 10, 0, 0),
                F.fire_mesh(128, 96, 6.0, 6.0, 0, 10, 0, 0), F.fire_mesh(128, 96, 6.0, 6.0, 10, 27, 0, 0),
                F.fire_mesh(128, 96, 6.0, 6.0, 10, 10, 7, 0)):
        assert lib.fire_state_bytes(C.byref(bad), 13) == 0
    assert lib.fire_state_bytes(C.byref(m), 0) == 0
    assert lib.fire_state_bytes(C.byref(m), 257) == 0
    assert lib.fire_abi_version() == 3
    assert lib.fire_strerror(-4) == b"fire reached the domain boundary guard ring"
    assert lib.fire_strerror(0) == b"ok"
    # argument errors are reported before any device work
    ctx = C.c_void_p()
    assert lib.fire_init(C.byref(ctx), None, None, 0, None, None, None, None, 0, None, None,
                         C.c_size_t(0), None) == -1
    assert lib.fire_step(None, None, None, C.c_double(0.5), None, None, None) == -1
    assert lib.fire_status(None) == -1


def test_ensemble_layout_and_errors_without_gpu(lib):
    from paper_1102_1343_amd import fire as F
    lib.fire_ens_state_bytes.restype = C.c_size_t
    sides = [(37, 50), (256, 300), (10, 10), (1001, 7)]
    ms = (F.fire_mesh * len(sides))(*[F.fire_mesh(nx, ny, 6.0, 6.0, 10, 10, F.FIRE_F32, 0)
                                      for nx, ny in sides])
    co = (C.c_int64 * (len(sides) + 1))()
    ao = (C.c_int64 * (len(sides) + 1))()
    assert lib.fire_ens_layout(ms, len(sides), co, ao) == 0
    cells = [0]
    atm = [0]
    for nx, ny in sides:
        cells.append(cells[-1] + nx * ny)
        atm.append(atm[-1] + -(-nx // 10) * -(-ny // 10))
    assert list(co) == cells and list(ao) == atm
    nb = lib.fire_ens_state_bytes(ms, len(sides), 13)
    assert nb >= 16 * cells[-1] + 2 * atm[-1]
    assert lib.fire_ens_state_bytes(ms, len(sides), 0) == 0
    # members must share dtype and refinement ratio
    for field, val in (("dtype", F.FIRE_F64), ("sr_x", 5), ("sr_y", 2)):
        bad = (F.fire_mesh * 2)(ms[0], ms[1])
        setattr(bad[1], field, val)
        assert lib.fire_ens_layout(bad, 2, co, ao) == -1
        assert lib.fire_ens_state_bytes(bad, 2, 13) == 0
    assert lib.fire_ens_layout(ms, 0, co, ao) == -1
    assert lib.fire_ens_layout(ms, 70000, co, ao) == -1
    h = C.c_void_p()
    nign = (C.c_int32 * len(sides))()
    assert lib.fire_ens_init(C.byref(h), ms, len(sides), None, 0, None, None, None, None, nign,
                             None, None, C.c_size_t(0), None) == -1
    assert lib.fire_ens_step(None, None, None, C.c_double(0.5), None, None) == -1
    assert lib.fire_ens_status(None, None) == -1


def test_adjoint_sizes_and_errors_without_gpu(lib):
    from paper_1102_1343_amd import fire as F
    lib.fire_adj_bytes.restype = C.c_size_t
    m = F.fire_mesh(100, 80, 6.0, 6.0, 10, 10, F.FIRE_F32, 0)
    n = 100 * 80
    nb = lib.fire_adj_bytes(C.byref(m), 13, 500, 50)
    # 10 checkpoints, two sets of replay buffers (51 levels of psi, 50 of
    # psi' and of psi* each), plus the working arrays
    assert nb >= (10 + 2 * 151) * 4 * n
    assert nb <= (10 + 2 * 151 + 40) * 4 * n
    assert lib.fire_adj_bytes(C.byref(m), 13, 0, 50) == 0
    assert lib.fire_adj_bytes(C.byref(m), 13, 500, 0) == 0
    assert lib.fire_adj_bytes(C.byref(m), 0, 500, 50) == 0
    h = C.c_void_p()
    assert lib.fire_adj_init(C.byref(h), None, 10, 5, None, C.c_size_t(0)) == -1
    assert lib.fire_adj_forward(None, None, None, C.c_double(0.25)) == -1
    assert lib.fire_adj_backward(None, None, None, None, None, None) == -1


def test_wind_grid_layout_and_errors_without_gpu(lib, tmp_path):
    from paper_1102_1343_amd import fire as F
    prog = tmp_path / "wg.c"
    prog.write_text('#include "fire.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                    'int main(void){printf("%zu %zu %zu\\n", sizeof(fire_wind_grid),'
                    'offsetof(fire_wind_grid, zf), offsetof(fire_wind_grid, g));return 0;}\n')
    exe = tmp_path / "wg"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got == [C.sizeof(F.fire_wind_grid), F.fire_wind_grid.zf.offset,
                   F.fire_wind_grid.g.offset]
    lib.fire_wind_scratch_bytes.restype = C.c_size_t
    g = F.fire_wind_grid(820, 820, 40, 10, 10, 8192, 8192, F.FIRE_F32, 6.1, 9.81)
    assert lib.fire_wind_scratch_bytes(C.byref(g)) >= (821 * 820 * 2) * 4
    for field, val in (("nx", 8201), ("ny", 0), ("nz", 0), ("zf", 0.0), ("g", -1.0),
                       ("dtype", 5), ("sr_x", 0)):
        b = F.fire_wind_grid(820, 820, 40, 10, 10, 8192, 8192, F.FIRE_F32, 6.1, 9.81)
        setattr(b, field, val)
        assert lib.fire_wind_scratch_bytes(C.byref(b)) == 0, field
    assert lib.fire_wind_interp(C.byref(g), None, None, None, None, None, None, None, None,
                                C.c_size_t(0), None) == -1


def test_static_wind_refuses_oversize_grid_without_gpu(lib):
    """The no-allocation coupling-input call checks the grid against its fixed
    scratch before any device call (the pointers are never touched)."""
    from paper_1102_1343_amd import fire as F
    lib.fire_wind_scratch_bytes.restype = C.c_size_t
    big = F.fire_wind_grid(1500, 1500, 1, 1, 1, 10, 10, F.FIRE_F32, 6.1, 9.81)
    assert lib.fire_wind_scratch_bytes(C.byref(big)) > F.WIND_STATIC_BYTES
    fake = [C.c_void_p(256)] * 7
    assert lib.fire_wind_interp_static(C.byref(big), *fake, None) == F.ERR_TOO_LARGE
    bad = F.fire_wind_grid(0, 1500, 1, 1, 1, 10, 10, F.FIRE_F32, 6.1, 9.81)
    assert lib.fire_wind_interp_static(C.byref(bad), *fake, None) == -1
    ok = F.fire_wind_grid(820, 820, 40, 10, 10, 8192, 8192, F.FIRE_F64, 6.1, 9.81)
    assert lib.fire_wind_scratch_bytes(C.byref(ok)) <= F.WIND_STATIC_BYTES
