"""Oracle: real 2D P_N moment matrices, grid classes and time step, in FP64.

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

Each function restates a definition of Seibold & Frank, "StaRMAP - A second
order staggered grid method for spherical harmonics moment equations of
radiative transfer" (arXiv 1211.2205):
  * moment list and order ............ Sect. 3 (2D reduction, transformation S)
  * complex matrices ................. Sect. 3, eq. (Pncomplex) x- and y-rows,
                                       recursion coefficients a..f
  * real matrices M = S M_c S^{-1} ... Sect. 3 (eq. transformation)
  * slab matrix ...................... Sect. 2 (eq. PN_slab)
  * grid classes ..................... Sect. 4.1 (eq. matrix_conditions) and
                                       the greedy assignment of Sect. 5.3
  * time step ........................ Sect. 4.5 (Thm. 1 and the rules after it)
"""
from __future__ import annotations

import math

import numpy as np


# ----------------------------------------------------------------- moments
def moments(N: int):
    """Real moments in the paper's order (Sect. 3, eq. transformation):
    l ascending; within l, m = l, l-2, ... >= 0 descending; R_l^m before I_l^m
    (I exists for m > 0 only).  Returns a list of (kind, l, m), kind in 'RI'."""
    out = []
    for l in range(N + 1):
        for m in range(l, -1, -2):
            out.append(("R", l, m))
            if m > 0:
                out.append(("I", l, m))
    return out


def complex_moments(N: int):
    """Complex moments psi_l^m kept by the 2D reduction (l + m even), in the
    paper's order psi_0^0, psi_1^-1, psi_1^1, psi_2^-2, psi_2^0, psi_2^2, ..."""
    return [(l, m) for l in range(N + 1) for m in range(-l, l + 1, 2)]


# ------------------------------------------------------ recursion coefficients
def coef_a(l, m):
    return math.sqrt((l - m + 1) * (l + m + 1) / ((2 * l + 3) * (2 * l + 1)))


def coef_b(l, m):
    return math.sqrt((l - m) * (l + m) / ((2 * l + 1) * (2 * l - 1)))


def coef_c(l, m):
    return math.sqrt((l + m + 1) * (l + m + 2) / ((2 * l + 3) * (2 * l + 1)))


def coef_d(l, m):
    return math.sqrt((l - m) * (l - m - 1) / ((2 * l + 1) * (2 * l - 1)))


def coef_e(l, m):
    return math.sqrt((l - m + 1) * (l - m + 2) / ((2 * l + 3) * (2 * l + 1)))


def coef_f(l, m):
    return math.sqrt((l + m) * (l + m - 1) / ((2 * l + 1) * (2 * l - 1)))


def _safe(fn, l, m):
    """A coefficient attached to a moment that does not exist (l < 0 or |m| > l)
    multiplies a vanishing term; return 0 there instead of evaluating the root of
    a possibly negative product."""
    if l < 0 or abs(m) > l:
        return 0.0
    return fn(l, m)


def complex_matrices(N: int):
    """M_x^complex (with the factor 1/2) and M_y^complex (with the factor i/2)
    from the x- and y-rows of eq. (Pncomplex).  Terms whose moment lies outside
    the kept set (l' > N: the P_N truncation; |m'| > l') are dropped."""
    cm = complex_moments(N)
    idx = {lm: i for i, lm in enumerate(cm)}
    n = len(cm)
    Mx = np.zeros((n, n), dtype=np.complex128)
    My = np.zeros((n, n), dtype=np.complex128)
    for (l, m), row in idx.items():
        # (target moment, x coefficient, y coefficient) of the row of psi_l^m
        terms = [
            ((l - 1, m - 1), -_safe(coef_c, l - 1, m - 1), +_safe(coef_c, l - 1, m - 1)),
            ((l + 1, m - 1), +_safe(coef_d, l + 1, m - 1), -_safe(coef_d, l + 1, m - 1)),
            ((l - 1, m + 1), +_safe(coef_e, l - 1, m + 1), +_safe(coef_e, l - 1, m + 1)),
            ((l + 1, m + 1), -_safe(coef_f, l + 1, m + 1), -_safe(coef_f, l + 1, m + 1)),
        ]
        for tgt, cx, cy in terms:
            col = idx.get(tgt)
            if col is None:
                continue
            Mx[row, col] += 0.5 * cx
            My[row, col] += 0.5j * cy
    return Mx, My


def transformation(N: int):
    """Unitary S with u = S psi (Sect. 3): R_l^0 = psi_l^0 and, for m > 0,
    R_l^m = (-1)^m/sqrt2 (psi^m + (-1)^m psi^-m),
    I_l^m = (-1)^m i/sqrt2 (psi^m - (-1)^m psi^-m)."""
    rm = moments(N)
    cidx = {lm: i for i, lm in enumerate(complex_moments(N))}
    S = np.zeros((len(rm), len(cidx)), dtype=np.complex128)
    r2 = 1.0 / math.sqrt(2.0)
    for row, (kind, l, m) in enumerate(rm):
        if m == 0:
            S[row, cidx[(l, 0)]] = 1.0
            continue
        sg = (-1.0) ** m
        if kind == "R":
            S[row, cidx[(l, m)]] = sg * r2
            S[row, cidx[(l, -m)]] = sg * sg * r2
        else:
            S[row, cidx[(l, m)]] = sg * 1j * r2
            S[row, cidx[(l, -m)]] = -sg * sg * 1j * r2
    return S


def real_matrices(N: int, clean: float = 1e-14):
    """M^real = S M^complex S^{-1} for x and y.  The products are real up to
    round-off; |imag| is asserted below `clean` and entries below `clean` in
    magnitude (exact zeros of the method, polluted by round-off) are set to 0."""
    Mxc, Myc = complex_matrices(N)
    S = transformation(N)
    Sinv = np.linalg.inv(S)
    out = []
    for Mc in (Mxc, Myc):
        M = S @ Mc @ Sinv
        assert np.max(np.abs(M.imag), initial=0.0) < clean, "real transform left an imaginary part"
        M = M.real.copy()
        M[np.abs(M) < clean] = 0.0
        out.append(M)
    return out[0], out[1]


def slab_matrix(N: int):
    """Slab-geometry P_N flux matrix (eq. PN_slab): row l couples to psi_{l-1}
    with l/(2l+1) and to psi_{l+1} with (l+1)/(2l+1); truncated at l = N."""
    M = np.zeros((N + 1, N + 1))
    for l in range(N + 1):
        if l > 0:
            M[l, l - 1] = l / (2 * l + 1)
        if l < N:
            M[l, l + 1] = (l + 1) / (2 * l + 1)
    return M


# ------------------------------------------------------------- grid classes
def grid_classes(Mx: np.ndarray, My: np.ndarray):
    """Greedy assignment of the components to the index sets I11, I21, I12, I22
    (Sect. 5.3): component 0 goes to I11; a nonzero Mx(i,j) puts j on the grid
    staggered in x from i's, a nonzero My(i,j) on the grid staggered in y.
    Returns arrays gx, gy with values 1 (cell centres) or 2 (nodes) per axis,
    i.e. component k lives on G_{gx[k] gy[k]}.  Asserts the result satisfies the
    nonzero conditions of eq. (matrix_conditions)."""
    n = Mx.shape[0]
    gx = np.zeros(n, dtype=np.int64)
    gy = np.zeros(n, dtype=np.int64)
    gx[0], gy[0] = 1, 1
    stack = [0]
    while stack:
        i = stack.pop()
        for j in np.nonzero(Mx[i])[0]:
            want = (3 - gx[i], gy[i])
            if gx[j] == 0:
                gx[j], gy[j] = want
                stack.append(j)
            assert (gx[j], gy[j]) == want, "M_x pattern violates the staggering conditions"
        for j in np.nonzero(My[i])[0]:
            want = (gx[i], 3 - gy[i])
            if gx[j] == 0:
                gx[j], gy[j] = want
                stack.append(j)
            assert (gx[j], gy[j]) == want, "M_y pattern violates the staggering conditions"
    assert np.all(gx > 0), "some component is not reached from the first one"
    return gx, gy


def is_even_component(gx, gy):
    """Even components: I11 and I22; odd components: I21 and I12 (Sect. 4.3)."""
    return np.asarray(gx) == np.asarray(gy)


# ---------------------------------------------------------------- time step
def spectral_radius(Mx: np.ndarray) -> float:
    """Largest eigenvalue magnitude of M_x (dense symmetric eigen-solver)."""
    return float(np.max(np.abs(np.linalg.eigvalsh(Mx))))


def time_step(cfl: float, dx: float, dy: float, rho: float, t_final: float):
    """dt0 = cfl * min(dx, dy) / rho (Thm. 1 scaled by 1/rho; the cfl number
    carries the 2D factor); the step count n lands exactly on t_final:
    n = ceil(t_final / dt0), dt = t_final / n."""
    dt0 = cfl * min(dx, dy) / rho
    n = int(math.ceil(t_final / dt0 - 1e-12))
    n = max(n, 1)
    return t_final / n, n


def direction_moments(N: int, omega):
    """Moments of a unit-weight beam delta(Omega - Omega_0): the real basis
    functions of the moment vector evaluated at Omega_0 = (ox, oy, oz).

    From the complex spherical harmonics Y_l^m (Sect. 3, with the usual
    Condon-Shortley phase; here scipy's sph_harm_y) the expansion coefficients
    of the delta are psi_l^m = conj(Y_l^m(Omega_0)); the change of variables
    to R_l^m, I_l^m (Sect. 3) gives R_l^0 = Y_l^0, R_l^m = (-1)^m sqrt2
    Re Y_l^m, I_l^m = (-1)^m sqrt2 Im Y_l^m."""
    from scipy.special import sph_harm_y
    ox, oy, oz = (float(v) for v in omega)
    polar = math.acos(max(-1.0, min(1.0, oz)))
    azim = math.atan2(oy, ox)
    out = []
    for kind, l, m in moments(N):
        y = complex(sph_harm_y(l, m, polar, azim))
        if m == 0:
            out.append(y.real)
        elif kind == "R":
            out.append((-1) ** m * math.sqrt(2.0) * y.real)
        else:
            out.append((-1) ** m * math.sqrt(2.0) * y.imag)
    return np.array(out)
