"""Oracle: the learned closure of the P_5 hierarchy, in plain FP64.

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

The P_N truncation drops the coupling of the top order to order N + 1 (Sect. 2:
the moment system is closed by setting the order-(N+1) moments to zero).  The
learned closure restores an estimate of the dropped flux of the order-5
moments,
    F_k = - sum_{j of order 6} ( Mx(k, j) D_x u_j + My(k, j) D_y u_j ),
from local order-4 and order-5 data, with a small network (oracle.mlp):

  * evaluation points: index pairs (i, j), 0 <= i <= nx, 0 <= j <= ny; the
    order-5 R moments (grid G21) take the outputs at their point (i, j) and
    the order-5 I moments (grid G12) at theirs, where those points exist;
  * inputs: for each of the eleven order-4/5 moments, in moment order, its
    values at the array neighbours (i + a, j + b), b = -1, 0, 1 (outer),
    a = -1, 0, 1 (inner), indices clamped to that moment's own array; then
    log10(sigma_a + 0.01) and log10(sigma_s + 0.01) at the G11 cell
    (min(i, nx - 1), min(j, ny - 1)); zeros up to 128 inputs;
  * scale equivariance (the equations are linear): the 99 moment inputs are
    divided by nu = sqrt(sum of their squares) + 1e-20, and the closure term
    of output r is g = nu * y_r / h, h = dx;
  * outputs, in moment order: R_5^5, I_5^5, R_5^3, I_5^3, R_5^1, I_5^1;
  * training target of output r at a point: F_k * h / nu.

The closure solver is the fused composition of the scheme, S^o_{dt/2},
[S^e_{dt}, S^o_{dt}]^(n-1), S^e_{dt}, S^o_{dt/2}, in which every odd sweep adds
g, evaluated on the state at the start of that sweep, to W_k of the order-5
rows (g is frozen during the sweep, as W is).
"""
from __future__ import annotations

import math

import numpy as np

from . import mlp, pn
from .scheme import OracleSolver

EPS = 1e-20
N_IN, N_HIDDEN, N_OUT = 128, 128, 6
N_FEATURES = 101


def closure_moments():
    """(kind, l, m) of the eleven input moments and the six output moments."""
    inputs = [km for km in pn.moments(5) if km[1] >= 4]
    outputs = [km for km in pn.moments(5) if km[1] == 5]
    return inputs, outputs


def _index_of(moms, key):
    return moms.index(key)


def sigma_features(sa, ss):
    return np.log10(sa + 0.01), np.log10(ss + 0.01)


def features(solver, points):
    """Inputs (count x 128) and norms nu (count) at the evaluation points
    [(i, j), ...] of a solver of order >= 5 (its order-4/5 moments are used)."""
    inputs, _ = closure_moments()
    g = solver.grid
    idx = [_index_of(solver.moms, km) for km in inputs]
    # sigma at the G11 cells
    X11, Y11 = g.coords(1, 1)
    sa = np.asarray(solver.prob.sigma_a(0.0, X11, Y11), dtype=np.float64) * np.ones(X11.shape)
    ss = np.asarray(solver.prob.sigma_s0(0.0, X11, Y11), dtype=np.float64) * np.ones(X11.shape)
    fa, fs = sigma_features(sa, ss)
    pts = np.asarray(points, dtype=np.int64).reshape(-1, 2)
    X = np.zeros((len(pts), N_IN))
    nu = np.zeros(len(pts))
    for r, (i, j) in enumerate(pts):
        vals = []
        for k in idx:
            a = solver.u[k]
            ny_k, nx_k = a.shape
            for b in (-1, 0, 1):
                jj = min(max(j + b, 0), ny_k - 1)
                for c in (-1, 0, 1):
                    ii = min(max(i + c, 0), nx_k - 1)
                    vals.append(a[jj, ii])
        v = np.array(vals)
        nu[r] = math.sqrt(float(np.sum(v * v))) + EPS
        X[r, :99] = v / nu[r]
        ci, cj = min(i, g.nx - 1), min(j, g.ny - 1)
        X[r, 99] = fa[cj, ci]
        X[r, 100] = fs[cj, ci]
    return X, nu


def order6_flux(solver):
    """F_k for every odd moment k of a solver of order >= 6: the odd residual W
    computed from the order-6 moments alone (all other planes zero)."""
    keep = [m[1] == 6 for m in solver.moms]
    saved = solver.u
    solver.u = [a if keep[k] else np.zeros_like(a) for k, a in enumerate(saved)]
    try:
        W = solver.flux(1)
    finally:
        solver.u = saved
    return W


def targets(solver, points, nu):
    """Training targets F_k h / nu at interior cells (i < nx, j < ny), where
    both the G21 and the G12 point (i, j) exist."""
    _, outputs = closure_moments()
    W = order6_flux(solver)
    h = solver.grid.dx
    pts = np.asarray(points, dtype=np.int64).reshape(-1, 2)
    T = np.zeros((len(pts), N_OUT))
    for r, (i, j) in enumerate(pts):
        for o, km in enumerate(outputs):
            k = _index_of(solver.moms, km)
            T[r, o] = W[k][j, i] * h / nu[r]
    return T


def closure_terms(solver, params, bf16=False):
    """g for the six order-5 moments of a P_5 solver, on their own grids."""
    g = solver.grid
    _, outputs = closure_moments()
    pts = [(i, j) for j in range(g.ny + 1) for i in range(g.nx + 1)]
    X, nu = features(solver, pts)
    Y, _ = mlp.forward(params, X, bf16=bf16)
    G = {}
    for o, km in enumerate(outputs):
        k = _index_of(solver.moms, km)
        shape = solver.u[k].shape
        full = (nu * Y[:, o] / g.dx).reshape(g.ny + 1, g.nx + 1)
        G[k] = np.ascontiguousarray(full[:shape[0], :shape[1]])
    return G


class ClosureSolver(OracleSolver):
    """P_5 oracle solver with the learned closure added to the odd sweeps."""

    def __init__(self, prob, params, bf16=False, **kw):
        assert prob.N == 5 and not prob.time_dependent
        super().__init__(prob, **kw)
        self.params = params
        self.bf16 = bf16

    def _odd(self, tau):
        G = closure_terms(self, self.params, self.bf16)
        W = self.flux(1)
        for k, gk in G.items():
            W[k] = W[k] + gk
        self.update(1, W, tau)

    def advance(self, nsteps, fused=True, callback=None):
        assert fused, "the closure solver is defined on the fused composition"
        if nsteps <= 0:
            return
        self._materials_for_step(self.t)
        dt = self.dt
        self._odd(0.5 * dt)
        for s in range(nsteps):
            self.half_step(0, dt)
            self._odd(dt if s < nsteps - 1 else 0.5 * dt)
        self.step_count += nsteps
        self.t = self.step_count * self.dt

    def run(self, fused=True):
        self.advance(self.nsteps - self.step_count, fused=True)


def r00_error(u00, ref00):
    """Relative L2 error of the zeroth moment on G11 (same grid)."""
    return math.sqrt(float(np.sum((u00 - ref00) ** 2)) / float(np.sum(ref00 ** 2)))
