"""Oracle side of the adjoint tests: the loss of a run computed with the FP64
oracle, and its central finite differences (the reference gradient)."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1102_1343_amd import synth


def shifted(ignitions, shift):
    return [dict(g, ax=g["ax"] + sx, ay=g["ay"] + sy, bx=g["bx"] + sx, by=g["by"] + sy)
            for g, (sx, sy) in zip(ignitions, shift)]


def run_F(prob, u, v, mult, shift, nsteps):
    """Fuel fraction after nsteps oracle steps under wind (u, v), per-category
    multipliers mult and ignitions translated by shift."""
    fuels = [dict(f, ros_mult=float(m)) for f, m in zip(prob.fuels, mult)]
    p = synth.Problem(prob.nx, prob.ny, prob.dx, prob.dy, prob.sr_x, prob.sr_y, fuels, prob.cat,
                      prob.dzdx, prob.dzdy, shifted(prob.ignitions, shift), prob.dt, nsteps,
                      [(u, v)], 0, dict(prob.params), prob.name)
    o = oracle.OracleFire(p)
    for _ in range(nsteps):
        o.step(u, v, p.dt)
    return o.frac.copy()


def loss(F, target):
    return 0.5 * float(np.sum((F - target) ** 2))


class Case:
    """A small adjoint case: problem, base parameters, oracle target."""

    def __init__(self, n, nsteps, seed=synth.SEED):
        prob, pert = synth.adjoint_case(n=n, steps=nsteps, seed=seed)
        self.prob, self.nsteps = prob, nsteps
        self.u, self.v = prob.wind[0]
        self.mult = np.ones(len(prob.fuels))
        self.shift = np.zeros((len(prob.ignitions), 2))
        s = pert["wind_scale"]
        self.target = run_F(prob, s * self.u, s * self.v, pert["mult"], pert["shift"], nsteps)

    def L(self, du=None, dv=None, mult=None, shift=None):
        u = self.u if du is None else self.u + du
        v = self.v if dv is None else self.v + dv
        m = self.mult if mult is None else mult
        sh = self.shift if shift is None else shift
        return loss(run_F(self.prob, u, v, m, sh, self.nsteps), self.target)

    def dF(self):
        return run_F(self.prob, self.u, self.v, self.mult, self.shift, self.nsteps) - self.target

    # central differences
    def fd_mult(self, k, h=1e-6):
        mp, mm = self.mult.copy(), self.mult.copy()
        mp[k] += h
        mm[k] -= h
        return (self.L(mult=mp) - self.L(mult=mm)) / (2 * h)

    def fd_shift(self, g, c, h=1e-5):
        sp, sm = self.shift.copy(), self.shift.copy()
        sp[g, c] += h
        sm[g, c] -= h
        return (self.L(shift=sp) - self.L(shift=sm)) / (2 * h)

    def fd_wind(self, du, dv, h=1e-6):
        return (self.L(du=h * du, dv=h * dv) - self.L(du=-h * du, dv=-h * dv)) / (2 * h)
