"""Adjoint of a run of fire steps through the C ABI (needs a GPU).

The reference gradient is the central finite difference of the FP64 oracle's
loss L = 1/2 sum (F_end - F_target)^2, F_target from an oracle run with
perturbed multipliers, wind and ignition centres.  The FP64 adjoint must
match it for every category multiplier, both coordinates of both ignition
shifts and random directions in the per-cell wind; the FP32 adjoint must
follow the FP64 one; gradients must not depend on the checkpoint interval;
the autograd wrapper must return the ABI's gradients.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_1102_1343_amd import fire as F

from adjoint_ref import Case
from parity import host

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _gpu_grads(case, dtype, every):
    p = case.prob
    fire = F.Fire.from_problem(p, dtype=dtype)
    adj = F.FireAdjoint(fire, case.nsteps, every)
    u = torch.from_numpy(case.u).to("cuda", dtype).contiguous()
    v = torch.from_numpy(case.v).to("cuda", dtype).contiguous()
    Fend = adj.forward(u, v, p.dt).clone()
    dF = (Fend - torch.from_numpy(case.target).to("cuda", dtype)).contiguous()
    gu, gv, gm, gs = adj.backward(dF)
    torch.cuda.synchronize()
    out = (host(gu), host(gv), gm.copy(), gs.copy(), host(Fend))
    adj.close()
    fire.close()
    return out


def _close(got, ref, rel, what):
    scale = max(np.max(np.abs(ref)), 1e-30)
    err = np.max(np.abs(np.asarray(got) - np.asarray(ref)))
    _log(f"{what}: max err {err:.3e} (scale {scale:.3e})")
    assert err <= rel * scale, what


@pytest.fixture(scope="module")
def case64():
    return Case(64, 60)


def test_adjoint_fp64_matches_oracle_fd(case64):
    case = case64
    gu, gv, gm, gs, Fend = _gpu_grads(case, torch.float64, every=25)
    assert np.max(np.abs(Fend - (case.dF() + case.target))) <= 1e-9
    assert (Fend < 1).sum() > 50
    fd_m = np.array([case.fd_mult(k) for k in range(len(gm))])
    _close(gm, fd_m, 1e-5, "dL/dm_k")
    assert np.count_nonzero(fd_m) >= 5
    fd_s = np.array([[case.fd_shift(g, c) for c in range(2)] for g in range(gs.shape[0])])
    _close(gs, fd_s, 1e-5, "dL/dshift")
    rng = np.random.default_rng(3)
    got, ref = [], []
    for _ in range(4):
        du = rng.normal(size=case.u.shape)
        dv = rng.normal(size=case.v.shape)
        got.append(float(np.sum(gu * du) + np.sum(gv * dv)))
        ref.append(case.fd_wind(du, dv))
    _close(got, ref, 1e-5, "dL/d(u,v) along random directions")
    # single cells where the wind gradient is largest
    k = int(np.argmax(np.abs(gu)))
    e = np.zeros_like(case.u)
    e.flat[k] = 1.0
    _close([gu.flat[k]], [case.fd_wind(e, np.zeros_like(e), h=1e-5)], 1e-4, "dL/du at one cell")


def test_adjoint_independent_of_checkpoint_interval(case64):
    for dtype in (torch.float64, torch.float32):
        ref = _gpu_grads(case64, dtype, every=case64.nsteps)
        for every in (1, 7):
            got = _gpu_grads(case64, dtype, every=every)
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), (dtype, every)


def test_adjoint_fp32_follows_fp64(case64):
    g64 = _gpu_grads(case64, torch.float64, every=20)
    g32 = _gpu_grads(case64, torch.float32, every=20)
    for name, a, b in zip(("du", "dv", "dm", "dshift"), g32[:4], g64[:4]):
        _close(a, b, 1e-3, f"fp32 vs fp64 {name}")


def test_adjoint_larger_mesh_against_oracle_fd():
    case = Case(160, 100, seed=77)
    gu, gv, gm, gs, Fend = _gpu_grads(case, torch.float64, every=30)
    assert (Fend < 1).sum() > 100
    k = int(np.argmax(np.abs(gm)))
    _close([gm[k]], [case.fd_mult(k)], 1e-5, f"dL/dm_{k} (160^2)")
    _close([gs[1, 0]], [case.fd_shift(1, 0)], 1e-5, "dL/dshift (160^2)")
    rng = np.random.default_rng(9)
    du = rng.normal(size=case.u.shape)
    dv = rng.normal(size=case.v.shape)
    _close([float(np.sum(gu * du) + np.sum(gv * dv))], [case.fd_wind(du, dv)], 1e-5,
           "dL/d(u,v) direction (160^2)")


def test_autograd_wrapper_matches_abi(case64):
    case = case64
    p = case.prob
    u = torch.from_numpy(case.u.copy()).cuda().requires_grad_(True)
    v = torch.from_numpy(case.v.copy()).cuda().requires_grad_(True)
    m = torch.ones(len(p.fuels), dtype=torch.float64, requires_grad=True)
    s = torch.zeros(len(p.ignitions), 2, dtype=torch.float64, requires_grad=True)
    Fend = F.FireRun.apply(u, v, m, s, p, case.nsteps, 25, torch.float64)
    L = 0.5 * ((Fend - torch.from_numpy(case.target).cuda()) ** 2).sum()
    L.backward()
    gu, gv, gm, gs, _ = _gpu_grads(case, torch.float64, every=25)
    assert np.array_equal(host(u.grad), gu)
    assert np.array_equal(host(v.grad), gv)
    assert np.array_equal(m.grad.numpy(), gm)
    assert np.array_equal(s.grad.numpy(), gs)
    assert abs(float(L.detach()) - case.L()) <= 1e-9 * abs(case.L())


def test_backward_after_more_steps_is_refused(case64):
    p = case64.prob
    fire = F.Fire.from_problem(p, dtype=torch.float64)
    adj = F.FireAdjoint(fire, 5, 5)
    u = torch.from_numpy(case64.u).cuda().contiguous()
    v = torch.from_numpy(case64.v).cuda().contiguous()
    adj.forward(u, v, p.dt)
    fire.step(u, v, p.dt)
    with pytest.raises(F.FireError) as ei:
        adj.backward(torch.zeros_like(u))
    assert ei.value.code == -6


def test_adjoint_every_cell_against_oracle_fd():
    """dL/du and dL/dv at every cell of a 20 x 20 case over 30 steps against
    central differences of the FP64 oracle's loss, one cell at a time."""
    case = Case(20, 30, seed=31)
    gu, gv, gm, gs, Fend = _gpu_grads(case, torch.float64, every=10)
    assert (Fend < 1).sum() > 40
    fu = np.zeros_like(gu)
    fv = np.zeros_like(gv)
    e = np.zeros_like(case.u)
    z = np.zeros_like(case.u)
    for k in range(e.size):
        e.flat[k] = 1.0
        fu.flat[k] = case.fd_wind(e, z, h=1e-6)
        fv.flat[k] = case.fd_wind(z, e, h=1e-6)
        e.flat[k] = 0.0
    for name, got, ref in (("dL/du", gu, fu), ("dL/dv", gv, fv)):
        scale = np.max(np.abs(ref))
        err = np.abs(got - ref)
        _log(f"{name} per cell: max err {err.max():.3e}, scale {scale:.3e}, "
             f"nonzero cells {np.count_nonzero(np.abs(ref) > 1e-6 * scale)}")
        assert np.count_nonzero(np.abs(ref) > 1e-3 * scale) >= 20
        assert err.max() <= 1e-5 * scale
