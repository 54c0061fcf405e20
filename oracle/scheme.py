"""Oracle: FP64 driver of the staggered-grid scheme (the paper's Sects. 4-5).

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

The time loop is the paper's literal composition (eq. solution_operator_full_step):
per step, evaluate materials and sources at t + dt/2 (once if time-independent,
Sect. 5.7), then S^o_{dt/2}, compute the even residual once, S^e_{dt/2} twice with
it (Sect. 5.8), recompute the odd residual, S^o_{dt/2}.  The optional `fused`
composition instead applies S^o_{dt/2}, [S^e_{dt}, S^o_{dt}]^(n-1), S^e_{dt},
S^o_{dt/2}; with frozen data both compositions are equal in exact arithmetic.

Two moment models of the paper's outlook (Sect. 7) use the same scheme:
  * filtered P_N (FP_N): per-order filter damping d_l added to the decay
    coefficient of every moment of order l (problem field `filter_damping`);
  * diffusion-corrected P_N (D_N): a diffusion step on the moments of the
    highest order, placed between the two even half-steps of every step:
    S^o_{dt/2} S^e_{dt/2} D_{dt} S^e_{dt/2} S^o_{dt/2}, with
    D_tau u = u + tau kappa (D_xx u + D_yy u) on each moment's own grid
    (three-point second differences; periodic axes wrap, extrapolation axes
    repeat the boundary value as ghost), explicit in time (problem field
    `diffusion` = kappa(x, y)).

Arrays follow the paper's index ranges per grid (cell index 1..n at (i-1/2)h,
node index p..n at i h; position 0 holds the first index), shape (rows, cols)
with x fastest.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import pn

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "starmap_oracle.c")
_LIB = os.path.join(_HERE, "_starmap_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fno-fast-math", "-ffp-contract=off",
               "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(dp)
        ip = ctypes.POINTER(ctypes.c_int)
        L.starmap_oracle_flux.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 2 + [
            ctypes.c_int, ip, ip, dp, dp, ctypes.c_int, pp, pp]
        L.starmap_oracle_update.argtypes = [ctypes.c_int] * 5 + [ip, ip, ctypes.c_int, pp, pp, pp, pp,
                                                                ctypes.c_double, ctypes.c_int]
        L.starmap_oracle_expm1div.argtypes = [ctypes.c_double, ctypes.c_int]
        L.starmap_oracle_expm1div.restype = ctypes.c_double
        L.starmap_oracle_set_threads.argtypes = [ctypes.c_int]
        L.starmap_oracle_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Thread count of the oracle's row loops (timing only; results do not
    depend on it).  Returns the count now in effect."""
    lib().starmap_oracle_set_threads(int(n))
    return lib().starmap_oracle_threads()


def threads() -> int:
    return lib().starmap_oracle_threads()


def expm1div(z: float, mode: int = 0) -> float:
    return lib().starmap_oracle_expm1div(float(z), int(mode))


def _ptrs(arrs):
    dp = ctypes.POINTER(ctypes.c_double)
    out = (dp * len(arrs))()
    for i, a in enumerate(arrs):
        if a is not None:
            assert a.dtype == np.float64 and a.flags.c_contiguous
            out[i] = a.ctypes.data_as(dp)
    return out


class Grid:
    """Staggered grids of a rectangle (eq. grid11, eq. staggered_grids)."""

    def __init__(self, n, ax, bc):
        self.nx, self.ny = int(n[0]), int(n[1])
        self.x0, self.x1, self.y0, self.y1 = map(float, ax)
        self.px = 1 if bc[0] == "periodic" else 0
        self.py = 1 if bc[1] == "periodic" else 0
        self.dx = (self.x1 - self.x0) / self.nx
        self.dy = (self.y1 - self.y0) / self.ny

    def axis(self, t, along_x):
        n, p, h, o = ((self.nx, self.px, self.dx, self.x0) if along_x
                      else (self.ny, self.py, self.dy, self.y0))
        if t == 1:
            i = np.arange(1, n + 1)
            return o + (i - 0.5) * h
        i = np.arange(p, n + 1)
        return o + i * h

    def shape(self, gx, gy):
        nxk = self.nx if gx == 1 else self.nx + 1 - self.px
        nyk = self.ny if gy == 1 else self.ny + 1 - self.py
        return (nyk, nxk)

    def coords(self, gx, gy):
        X, Y = np.meshgrid(self.axis(gx, True), self.axis(gy, False))
        return X, Y


class OracleSolver:
    """The staggered-grid P_N solver of the paper, for one problem
    (see workloads.Problem)."""

    def __init__(self, prob, emode: int = 0, moment_matrices=None):
        self.prob = prob
        self.N = prob.N
        self.moms = pn.moments(self.N)
        self.nmom = len(self.moms)
        if moment_matrices is None:
            self.Mx, self.My = pn.real_matrices(self.N)
        else:
            self.Mx, self.My = moment_matrices
        gx, gy = pn.grid_classes(self.Mx, self.My)
        self.gx = np.ascontiguousarray(gx, dtype=np.int32)
        self.gy = np.ascontiguousarray(gy, dtype=np.int32)
        self.grid = Grid(prob.n, prob.ax, prob.bc)
        self.rho = pn.spectral_radius(self.Mx)
        self.dt, self.nsteps = pn.time_step(prob.cfl, self.grid.dx, self.grid.dy, self.rho, prob.t_final)
        self.emode = emode
        self.t = 0.0
        self.step_count = 0
        self.u = []
        for k in range(self.nmom):
            X, Y = self.grid.coords(self.gx[k], self.gy[k])
            f = prob.initial.get(k)
            self.u.append(np.ascontiguousarray(f(0.0, X, Y) if f else np.zeros(X.shape), dtype=np.float64))
        self._mat_t = None
        self._c = self._q = None
        self._Mxc = np.ascontiguousarray(self.Mx)
        self._Myc = np.ascontiguousarray(self.My)

    # ------------------------------------------------------------ materials
    def evaluate_materials(self, t):
        """Decay c_k and source q_k on each component's grid at time t:
        c = sigma_a for the zeroth moment, c = sigma_a + sigma_s0 - sigma_sl for
        order l >= 1 (Sect. 2: Sigma_tl; Sect. 5.5); q only on the components the
        problem lists."""
        prob = self.prob
        c, q = [], []
        cache = {}
        any_q = False
        # a beam source q(x) delta(Omega - Omega_0) has moments q(x) phi_k(Omega_0)
        beam = None
        if getattr(prob, "beam_direction", None) is not None:
            beam = pn.direction_moments(self.N, prob.beam_direction)
        for k, (kind, l, m) in enumerate(self.moms):
            g = (int(self.gx[k]), int(self.gy[k]))
            if g not in cache:
                X, Y = self.grid.coords(*g)
                cache[g] = (X, Y, np.asarray(prob.sigma_a(t, X, Y), dtype=np.float64) * np.ones(X.shape),
                            np.asarray(prob.sigma_s0(t, X, Y), dtype=np.float64) * np.ones(X.shape))
            X, Y, sa, s0 = cache[g]
            if k == 0:
                ck = sa
            else:
                ck = sa + s0
                if prob.sigma_sl is not None:
                    ck = ck - np.asarray(prob.sigma_sl(l, t, X, Y), dtype=np.float64) * np.ones(X.shape)
            damping = getattr(prob, "filter_damping", None)
            if damping is not None:  # FP_N: the filter's damping of order l
                ck = ck + float(damping[l])
            c.append(np.ascontiguousarray(ck))
            f = prob.source.get(k)
            if f is None and beam is not None and beam[k] != 0.0:
                f = (lambda c: (lambda tt, xx, yy: c * prob.beam_profile(tt, xx, yy)))(float(beam[k]))
            if f is not None:
                q.append(np.ascontiguousarray(np.asarray(f(t, X, Y), dtype=np.float64) * np.ones(X.shape)))
                any_q = True
            else:
                q.append(None)
        self._c, self._q = c, (q if any_q else None)

    # ---------------------------------------------------------- operators
    def _alloc_w(self, parity):
        W = [None] * self.nmom
        for k in range(self.nmom):
            even = self.gx[k] == self.gy[k]
            if (parity == 0) == even:
                W[k] = np.zeros(self.grid.shape(self.gx[k], self.gy[k]))
        return W

    def flux(self, parity):
        """Residual W of the given parity (0 even, 1 odd) from the frozen other parity."""
        g = self.grid
        W = self._alloc_w(parity)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        st = lib().starmap_oracle_flux(
            g.nx, g.ny, g.px, g.py, g.dx, g.dy, self.nmom,
            self.gx.ctypes.data_as(ip), self.gy.ctypes.data_as(ip),
            self._Mxc.ctypes.data_as(dp), self._Myc.ctypes.data_as(dp),
            parity, _ptrs(self.u), _ptrs(W))
        assert st == 0, "coupling outside the staggering pattern"
        return W

    def update(self, parity, W, tau):
        g = self.grid
        ip = ctypes.POINTER(ctypes.c_int)
        q = self._q
        qp = _ptrs(q) if q is not None else None
        lib().starmap_oracle_update(
            g.nx, g.ny, g.px, g.py, self.nmom,
            self.gx.ctypes.data_as(ip), self.gy.ctypes.data_as(ip),
            parity, _ptrs(self.u), _ptrs(W), _ptrs(self._c), qp, float(tau), self.emode)

    def half_step(self, parity, tau, W=None):
        """S^parity_tau (eq. solution_operator_even / _odd)."""
        if W is None:
            W = self.flux(parity)
        self.update(parity, W, tau)
        return W

    def _materials_for_step(self, t):
        if self.prob.time_dependent or self._c is None:
            self.evaluate_materials(t + 0.5 * self.dt)

    def diffuse(self, tau):
        """D_N diffusion step on every moment of order N: u <- u + tau kappa
        (second difference along x / dx^2 + along y / dy^2), the differences
        taken on the moment's own grid; a periodic axis wraps, an
        extrapolation axis repeats the boundary point as its ghost."""
        g = self.grid
        for k, (kind, l, m) in enumerate(self.moms):
            if l != self.N:
                continue
            X, Y = g.coords(self.gx[k], self.gy[k])
            kap = np.asarray(self.prob.diffusion(0.0, X, Y), dtype=np.float64) * np.ones(X.shape)
            u = self.u[k]
            if g.px:
                east, west = np.roll(u, -1, axis=1), np.roll(u, 1, axis=1)
            else:
                east = np.concatenate([u[:, 1:], u[:, -1:]], axis=1)
                west = np.concatenate([u[:, :1], u[:, :-1]], axis=1)
            if g.py:
                north, south = np.roll(u, -1, axis=0), np.roll(u, 1, axis=0)
            else:
                north = np.concatenate([u[1:, :], u[-1:, :]], axis=0)
                south = np.concatenate([u[:1, :], u[:-1, :]], axis=0)
            lap = (east - 2.0 * u + west) / (g.dx * g.dx) + (north - 2.0 * u + south) / (g.dy * g.dy)
            self.u[k] = np.ascontiguousarray(u + tau * kap * lap)

    def step(self):
        """One full step t -> t + dt: S^o_{dt/2} S^e_{dt/2} S^e_{dt/2} S^o_{dt/2}
        (with a D_N diffusion step D_dt between the two even half-steps)."""
        h = 0.5 * self.dt
        self._materials_for_step(self.t)
        self.half_step(1, h)
        We = self.flux(0)
        self.half_step(0, h, We)
        if getattr(self.prob, "diffusion", None) is not None:
            self.diffuse(self.dt)
            We = None  # the diffusion changed moments the even residual reads
        self.half_step(0, h, We)
        self.half_step(1, h)
        self.step_count += 1
        self.t = self.step_count * self.dt

    def advance(self, nsteps, fused=False, callback=None):
        """Advance nsteps steps.  fused=True merges the two even half-steps into
        S^e_{dt} and the odd half-steps of consecutive steps into S^o_{dt}
        (time-independent problems only)."""
        if nsteps <= 0:
            return
        if not fused:
            for _ in range(nsteps):
                self.step()
                if callback is not None:
                    callback(self)
            return
        assert not self.prob.time_dependent
        assert getattr(self.prob, "diffusion", None) is None, "the D_N step splits the even half-steps"
        self._materials_for_step(self.t)
        dt = self.dt
        self.half_step(1, 0.5 * dt)
        for s in range(nsteps):
            self.half_step(0, dt)
            self.half_step(1, dt if s < nsteps - 1 else 0.5 * dt)
        self.step_count += nsteps
        self.t = self.step_count * self.dt

    def run(self, fused=False):
        self.advance(self.nsteps - self.step_count, fused=fused)

    # -------------------------------------------------------- diagnostics
    def mass(self):
        """dx dy * sum of the zeroth moment over G11."""
        return self.grid.dx * self.grid.dy * float(np.sum(self.u[0]))

    def l2(self):
        """Discrete L2 norm (dx dy sum_k sum u_k^2)^(1/2) (eq. discrete_L2_norm, 2D)."""
        s = sum(float(np.sum(a * a)) for a in self.u)
        return math.sqrt(self.grid.dx * self.grid.dy * s)
