"""Pins of the oracle's time stepping against closed forms, invariants and
brute force (Seibold & Frank, Sects. 4 and 6)."""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as wl
from oracle import pn
from oracle.scheme import OracleSolver, expm1div


def _const(v):
    return lambda t, x, y: np.full(np.broadcast(x, y).shape, float(v))


def _problem(N, n, ax, bc, sa, ss, cfl=0.5, t_final=0.3, initial=None, source=None, sigma_sl=None,
             time_dependent=False):
    return wl.Problem(name="t", N=N, n=n, ax=ax, bc=bc, cfl=cfl, t_final=t_final,
                      sigma_a=sa if callable(sa) else _const(sa),
                      sigma_s0=ss if callable(ss) else _const(ss), sigma_sl=sigma_sl,
                      initial=initial or {}, source=source or {}, time_dependent=time_dependent)


PER = ("periodic", "periodic")
EXT = ("extrapolation", "extrapolation")


# ------------------------------------------------------------------ E(z)
def test_expm1div():
    for z in (-50.0, -3.0, -1e-3, -2e-4, -1e-9, 0.0, 1e-9, 2e-4, 1e-3, 2.0):
        ref = 1.0 if z == 0 else math.expm1(z) / z
        assert abs(expm1div(z, 0) - ref) <= 2e-16 * abs(ref)
    # the paper's switched evaluation stays below 1e-12 total error (Sect. 5.6)
    for z in np.concatenate([np.linspace(-3e-4, 3e-4, 601), -np.logspace(-12, -1, 50)]):
        ref = 1.0 if z == 0 else math.expm1(z) / z
        assert abs(expm1div(float(z), 1) - ref) < 1e-12


# ---------------------------------------------------- single-cell closed form
@pytest.mark.parametrize("bc", [PER, EXT])
def test_uniform_state_follows_exact_ode(bc):
    """Uniform fields: all differences vanish and every component obeys
    u' = q - c u exactly (eq. sub_step_solution_division), with c = sigma_a for
    R_0^0 and sigma_a + sigma_s0 - sigma_sl for order l (Sect. 2)."""
    N, sa, ss, q0 = 3, 0.7, 1.3, 2.0
    u0 = {k: _const(0.1 * (k + 1)) for k in range(10)}
    prob = _problem(N, (6, 5), (0, 1, 0, 2), bc, sa, ss, t_final=0.9, initial=u0,
                    source={0: _const(q0)}, sigma_sl=lambda l, t, x, y: 0.6 ** l + 0 * x)
    o = OracleSolver(prob)
    o.run()
    t = prob.t_final
    for k, (kind, l, m) in enumerate(o.moms):
        c = sa if k == 0 else sa + ss - 0.6 ** l
        q = q0 if k == 0 else 0.0
        exact = math.exp(-c * t) * 0.1 * (k + 1) + (1 - math.exp(-c * t)) * q / c
        np.testing.assert_allclose(o.u[k], exact, rtol=1e-13)


def test_pure_absorption_decay():
    """Homogeneous pure absorption: R00(t) = R00(0) exp(-sigma_a t)."""
    prob = _problem(5, (8, 8), (-1, 1, -1, 1), EXT, 2.5, 0.0, t_final=1.0, initial={0: _const(3.0)})
    o = OracleSolver(prob)
    o.run()
    np.testing.assert_allclose(o.u[0], 3.0 * math.exp(-2.5), rtol=1e-13)
    for k in range(1, o.nmom):
        assert np.max(np.abs(o.u[k])) == 0.0


# ------------------------------------------------------------ conservation
def test_mass_conserved_periodic_without_absorption():
    """sigma_a = 0, q = 0, periodic: dx dy sum R00 is constant."""
    rng = np.random.default_rng(5)
    prob = _problem(5, (24, 20), (0, 1.2, 0, 1), PER, 0.0, 0.8, t_final=0.6)
    o = OracleSolver(prob)
    for k in range(o.nmom):
        o.u[k][:] = rng.standard_normal(o.u[k].shape)
    m0 = o.mass()
    o.run()
    assert abs(o.mass() - m0) < 1e-13 * max(1.0, abs(m0)) * 10


def test_periodic_semidiscrete_operator_is_skew():
    """The periodic operator -(M_x D_x + M_y D_y), assembled column by column
    from unit vectors, is skew-symmetric (brute force on a 4x3 grid)."""
    prob = _problem(3, (4, 3), (0, 1, 0, 0.6), PER, 0.0, 0.0)
    o = OracleSolver(prob)
    sizes = [a.size for a in o.u]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    n = offs[-1]
    L = np.zeros((n, n))
    for col in range(n):
        for k in range(o.nmom):
            o.u[k][:] = 0.0
        k = np.searchsorted(offs, col, side="right") - 1
        o.u[k].flat[col - offs[k]] = 1.0
        for parity in (0, 1):
            W = o.flux(parity)
            for kk, w in enumerate(W):
                if w is not None:
                    L[offs[kk]:offs[kk + 1], col] += w.ravel()
    assert np.max(np.abs(L)) > 1.0
    np.testing.assert_allclose(L, -L.T, atol=1e-15 * np.max(np.abs(L)) * 10)


# ----------------------------------------------- exact discrete Fourier law
def _growth(Mx, My, gx, gy, c, kx, ky, dx, dy, dt):
    """Amplification matrix of one full step for the mode exp(i(kx x + ky y)),
    built from the half-step operators: a_k <- exp(-c_k tau) a_k
    + tau E(-c_k tau) sum_j A_kj a_j with A = -(M_x sx + M_y sy),
    sx = (2i/dx) sin(kx dx / 2) (Sect. 4.5), G = G^o G^e G^e G^o."""
    n = len(c)
    sx = 2j / dx * math.sin(kx * dx / 2)
    sy = 2j / dy * math.sin(ky * dy / 2)
    A = -(Mx * sx + My * sy)

    def half(parity, tau):
        G = np.eye(n, dtype=complex)
        for k in range(n):
            even = gx[k] == gy[k]
            if (parity == 0) == even:
                z = -c[k] * tau
                E = 1.0 if z == 0 else math.expm1(z) / z
                G[k, :] = tau * E * A[k, :]
                G[k, k] = math.exp(z)
        return G

    h = 0.5 * dt
    return half(1, h) @ half(0, h) @ half(0, h) @ half(1, h)


@pytest.mark.parametrize("N,modes", [(1, (1, 0)), (3, (2, 1)), (5, (1, 3)), (4, (3, 2))])
def test_exact_discrete_fourier_evolution(N, modes):
    """Periodic, constant materials, one Fourier mode: the scheme's output equals
    G^n a0 exactly (up to round-off)."""
    Lx, Ly, nx, ny = 1.0, 1.5, 14, 12
    kx, ky = 2 * math.pi * modes[0] / Lx, 2 * math.pi * modes[1] / Ly
    sa, ss = 0.4, 0.9
    sl = lambda l, t, x, y: 0.5 ** l + 0 * x
    prob = _problem(N, (nx, ny), (0, Lx, 0, Ly), PER, sa, ss, t_final=0.7, sigma_sl=sl)
    o = OracleSolver(prob)
    rng = np.random.default_rng(N)
    a0 = rng.standard_normal(o.nmom) + 1j * rng.standard_normal(o.nmom)
    coords = [o.grid.coords(o.gx[k], o.gy[k]) for k in range(o.nmom)]
    for k in range(o.nmom):
        X, Y = coords[k]
        o.u[k][:] = (a0[k] * np.exp(1j * (kx * X + ky * Y))).real
    c = np.array([sa if k == 0 else sa + ss - 0.5 ** l for k, (_, l, _) in enumerate(o.moms)])
    G = _growth(o.Mx, o.My, o.gx, o.gy, c, kx, ky, o.grid.dx, o.grid.dy, o.dt)
    o.run()
    an = np.linalg.matrix_power(G, o.nsteps) @ a0
    scale = max(np.max(np.abs(a)) for a in o.u)
    for k in range(o.nmom):
        X, Y = coords[k]
        exp_k = (an[k] * np.exp(1j * (kx * X + ky * Y))).real
        np.testing.assert_allclose(o.u[k], exp_k, rtol=0, atol=1e-12 * scale)


def test_p1_growth_matrix_matches_paper_formula():
    """For P_1 in 1D the paper prints G (eq. growth_factor); the half-step
    products above reproduce it with the coupling coefficient 1/sqrt3."""
    Mx, My = pn.real_matrices(1)
    gx, gy = pn.grid_classes(Mx, My)
    ce, co, h, dt, k = 0.3, 1.1, 0.1, 0.04, 7.0
    G = _growth(Mx, My, gx, gy, np.array([ce, co, co]), k, 0.0, h, h, dt)
    a = Mx[0, 1]
    de, do = math.exp(-0.5 * ce * dt), math.exp(-0.5 * co * dt)
    Ee = math.expm1(-0.5 * ce * dt) / (-0.5 * ce * dt)
    Eo = math.expm1(-0.5 * co * dt) / (-0.5 * co * dt)
    fe = -1j * a * dt / h * Ee * math.sin(k * h / 2)
    fo = -1j * a * dt / h * Eo * math.sin(k * h / 2)
    Gp = np.array([[de ** 2 + (de + 1) * fe * fo, do * (de + 1) * fe],
                   [(do + de ** 2) * fo + (de + 1) * fe * fo ** 2, do ** 2 + do * (de + 1) * fe * fo]])
    np.testing.assert_allclose(G[:2, :2], Gp, atol=1e-15)


# ------------------------------------------------------ continuum telegraph
def test_p1_telegraph_second_order():
    """P_1 plane wave against the continuum solution exp(-t [[sa, i k/sqrt3],
    [i k/sqrt3, sa+ss]]) a0: the error falls by ~4 per halving of h."""
    sa, ss, T = 0.2, 0.5, 0.5
    kx = 2 * math.pi
    a0 = np.array([1.0, -0.3j])
    A = np.array([[sa, 1j * kx / math.sqrt(3)], [1j * kx / math.sqrt(3), sa + ss]])
    aT = scipy.linalg.expm(-T * A) @ a0
    errs = []
    for nx in (16, 32, 64, 128):
        init = {0: lambda t, x, y: np.cos(kx * x) + 0 * y, 1: lambda t, x, y: 0.3 * np.sin(kx * x) + 0 * y}
        prob = _problem(1, (nx, 2), (0, 1, 0, 2.0 / nx), PER, sa, ss, t_final=T, initial=init)
        o = OracleSolver(prob)
        o.run()
        e = 0.0
        for k in (0, 1):
            X, Y = o.grid.coords(o.gx[k], o.gy[k])
            e = max(e, np.max(np.abs(o.u[k] - (aT[k] * np.exp(1j * kx * X)).real)))
        assert np.max(np.abs(o.u[2])) == 0.0
        errs.append(e)
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.6 < r < 4.4 for r in ratios[1:]), ratios


# ---------------------------------------------------------------- stability
def test_stability_cfl():
    """cfl = 0.5 stays bounded; cfl = 0.72 (beyond the 2D limit 1/sqrt2) grows."""
    rho = pn.spectral_radius(pn.real_matrices(3)[0])

    def run(cfl):
        # 40 steps of exactly dt = cfl h / rho (t_final chosen so that no
        # shortening of dt to land on t_final takes place)
        t_final = 40 * cfl * (1.0 / 32) / rho
        prob = _problem(3, (32, 32), (0, 1, 0, 1), PER, 0.0, 0.0, cfl=cfl, t_final=t_final)
        o = OracleSolver(prob)
        rng = np.random.default_rng(1)
        for k in range(o.nmom):
            o.u[k][:] = rng.standard_normal(o.u[k].shape)
        l0 = o.l2()
        o.run()
        return o.l2() / l0
    assert run(0.5) < 2.0
    assert run(0.72) > 1e3


# ------------------------------------------------------ manufactured solution
def test_mms_second_order():
    """Manufactured solution of Sect. 6.1 (P_3, [0,1]^2 periodic, t <= 0.5,
    Sigma_a = t cos(2 pi y), Sigma_sl = 0.9^l, R00 = e^-t sin^2(2 pi x), all
    other moments zero).  Its source: q_R00 = R00 (Sigma_a - 1) and
    q_R11 = Mx(R11,R00) d/dx R00 with Mx(R11,R00) = sqrt2 d_1^-1 / 2 = 1/sqrt3
    (printed P_3 matrix); all other components vanish."""
    m_r11_r00 = math.sqrt(2.0) * math.sqrt(2.0 / 3.0) / 2.0
    sa = lambda t, x, y: t * np.cos(2 * math.pi * y) + 0 * x
    sl = lambda l, t, x, y: 0.9 ** l + 0 * x
    exact = lambda t, x, y: math.exp(-t) * np.sin(2 * math.pi * x) ** 2 + 0 * y
    q0 = lambda t, x, y: exact(t, x, y) * (t * np.cos(2 * math.pi * y) - 1.0)
    q1 = lambda t, x, y: m_r11_r00 * 2 * math.pi * math.exp(-t) * np.sin(4 * math.pi * x) + 0 * y
    errs = []
    for n in (16, 32, 64, 128):
        prob = _problem(3, (n, n), (0, 1, 0, 1), PER, sa, 1.0, t_final=0.5, initial={0: exact},
                        source={0: q0, 1: q1}, sigma_sl=sl, time_dependent=True)
        o = OracleSolver(prob)
        o.run()
        e2 = 0.0
        for k in range(o.nmom):
            X, Y = o.grid.coords(o.gx[k], o.gy[k])
            ref = exact(0.5, X, Y) if k == 0 else 0.0
            e2 += np.sum((o.u[k] - ref) ** 2)
        errs.append(math.sqrt(e2 * o.grid.dx * o.grid.dy))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert abs(orders[-1] - 2.0) < 0.15, (errs, orders)
    assert abs(orders[-2] - 2.0) < 0.25, (errs, orders)


def test_separable_manufactured_problem_is_the_paper_setting():
    """The time-separable form of the manufactured problem (terms a(t) g(x, y))
    gives the fields of Sect. 6.1 as written out above, and the oracle run on
    it ends within the second-order error of the exact solution."""
    prob = wl.manufactured(32)
    rng = np.random.Generator(np.random.PCG64(5))
    x, y = rng.uniform(0, 1, 50), rng.uniform(0, 1, 50)
    c = math.sqrt(2.0) * math.sqrt(2.0 / 3.0) / 2.0
    for t in (0.0, 0.13, 0.5):
        r00 = math.exp(-t) * np.sin(2 * math.pi * x) ** 2
        sa = t * np.cos(2 * math.pi * y)
        for f, ref in ((prob.sigma_a, sa), (prob.source[0], r00 * (sa - 1.0)),
                       (prob.source[1], c * 2 * math.pi * math.exp(-t) * np.sin(4 * math.pi * x))):
            np.testing.assert_allclose(f(t, x, y), ref, rtol=1e-14, atol=1e-14)
        for key, terms in (("absorption", prob.separable["absorption"]),
                           ("source0", prob.separable["source"][0]), ("source1", prob.separable["source"][1])):
            f = {"absorption": prob.sigma_a, "source0": prob.source[0], "source1": prob.source[1]}[key]
            np.testing.assert_allclose(sum(a(t) * g(x, y) for a, g in terms), f(t, x, y), rtol=1e-14, atol=1e-14)
    o = OracleSolver(prob)
    o.run()
    X, Y = o.grid.coords(o.gx[0], o.gy[0])
    err = np.sqrt(np.sum((o.u[0] - math.exp(-0.5) * np.sin(2 * math.pi * X) ** 2) ** 2) * o.grid.dx * o.grid.dy)
    assert err < 2.5e-3, err  # 1.84e-3 at 32^2, a quarter of it at 64^2


# ------------------------------------------------------ discrete L2 variation
def test_l2_norm_variation_small():
    """P_5 Gaussian (pseudo-time 1e-2) in a periodic void on [-1,1]^2 to t = 0.5:
    the discrete L2 norm varies by less than 0.02% at 100^2 (Sect. 6.2) and
    less at 200^2 than at 100^2."""
    var = {}
    for n in (50, 100, 200):
        prob = _problem(5, (n, n), (-1, 1, -1, 1), PER, 0.0, 0.0, t_final=0.5,
                        initial={0: wl.gaussian_pseudo_time(1e-2)})
        o = OracleSolver(prob)
        l0 = o.l2()
        dev = [0.0]
        o.advance(o.nsteps, callback=lambda s: dev.append(abs(s.l2() / l0 - 1.0)))
        var[n] = max(dev)
    assert var[100] < 2e-4, var
    assert var[200] < var[100], var


# ------------------------------------------------------------- symmetries
def test_line_source_reflection_symmetry():
    """Symmetric line source: R00 is symmetric under x<->y and x -> -x; every
    component maps by the signed permutation of the x<->y swap."""
    prob = wl.line_source(N=3, n=40, s=0.15, t_final=0.5)
    o = OracleSolver(prob)
    o.run()
    r = o.u[0]
    sc = np.max(np.abs(r))
    np.testing.assert_allclose(r, r.T, atol=1e-14 * sc)
    np.testing.assert_allclose(r, r[:, ::-1], atol=1e-14 * sc)
    np.testing.assert_allclose(r, r[::-1, :], atol=1e-14 * sc)
    idx = {t: i for i, t in enumerate(o.moms)}
    for k, (kind, l, m) in enumerate(o.moms):
        if m % 2 == 0:
            s = (-1.0) ** (m // 2) * (1 if kind == "R" else -1)
            j = k
        else:
            s = (-1.0) ** ((m - 1) // 2)
            j = idx[("I" if kind == "R" else "R", l, m)]
        np.testing.assert_allclose(o.u[k].T, s * o.u[j], atol=1e-14 * sc)


# ------------------------------------------------------------ fused steps
def test_fused_composition_equals_literal():
    """S^e_{dt/2} S^e_{dt/2} = S^e_{dt} and merged odd half-steps: the fused
    sequence equals the paper's four half-steps per step to round-off."""
    prob = wl.checkerboard(N=3, n=42, t_final=0.8)
    a = OracleSolver(prob)
    b = OracleSolver(prob)
    a.run(fused=False)
    b.run(fused=True)
    num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(a.u, b.u))
    den = sum(float(np.sum(x ** 2)) for x in a.u)
    assert math.sqrt(num / den) < 1e-13


# ------------------------------------------------ FP_N and D_N (Sect. 7 outlook)
@pytest.mark.parametrize("k", [0, 3, 9, 14])
def test_filter_damping_decays_a_uniform_moment_exactly(k):
    """A spatially uniform moment has zero differences, so each half-step
    multiplies it by exp(-c tau) exactly: with filter damping d_l the decay
    rate of an order-l moment is sigma_a + sigma_s0 + d_l (l >= 1), or
    sigma_a + d_0 for the zeroth moment."""
    N = 4
    l = pn.moments(N)[k][1]
    d = wl.filter_damping(N, 7.0, power=2)
    d[0] = 0.3
    prob = _problem(N, (12, 10), (0, 1, 0, 2), PER, 0.25, 1.5, t_final=0.4, initial={k: _const(2.0)})
    prob.filter_damping = d
    o = OracleSolver(prob)
    o.run()
    rate = 0.25 + d[0] if l == 0 else 0.25 + 1.5 + d[l]
    exact = 2.0 * math.exp(-rate * 0.4)
    np.testing.assert_allclose(o.u[k], exact, rtol=1e-13)
    for j in range(o.nmom):
        if j != k:
            assert np.max(np.abs(o.u[j])) < 1e-14
    # and damping zero reproduces plain P_N exactly
    prob.filter_damping = [0.0] * (N + 1)
    a = OracleSolver(prob)
    a.run()
    prob.filter_damping = None
    b = OracleSolver(prob)
    b.run()
    for x, y in zip(a.u, b.u):
        assert np.array_equal(x, y)


def _order_n_moments(o):
    return [k for k, (_, l, _) in enumerate(o.moms) if l == o.N]


@pytest.mark.parametrize("n", [(16, 12), (15, 20)])
def test_diffusion_step_has_the_discrete_fourier_symbol(n):
    """On a periodic grid a Fourier mode is an eigenvector of the three-point
    second difference: D_tau multiplies exp(i(a x + b y)) by
    1 - tau kappa (4/dx^2 sin^2(a dx/2) + 4/dy^2 sin^2(b dy/2)), on cell and
    nodal grids alike."""
    kappa = 0.01
    prob = _problem(3, n, (0, 1, 0, 1.5), PER, 0.0, 0.0, t_final=0.1)
    prob.diffusion = _const(kappa)
    o = OracleSolver(prob)
    ks = _order_n_moments(o)
    a, b = 2 * math.pi * 3, 2 * math.pi * 2 / 1.5
    for k in ks:
        X, Y = o.grid.coords(o.gx[k], o.gy[k])
        o.u[k] = np.ascontiguousarray(np.cos(a * X + b * Y))
    tau = 0.7 * o.dt
    o.diffuse(tau)
    g = o.grid
    lam = 1 - tau * kappa * (4 / g.dx ** 2 * math.sin(a * g.dx / 2) ** 2 + 4 / g.dy ** 2 * math.sin(b * g.dy / 2) ** 2)
    for k in ks:
        X, Y = o.grid.coords(o.gx[k], o.gy[k])
        np.testing.assert_allclose(o.u[k], lam * np.cos(a * X + b * Y), rtol=0, atol=1e-13)


def test_diffusion_step_conserves_cell_sums_and_constants():
    """With repeated-boundary ghosts the second difference of a cell-centred
    plane sums to zero (no flux through the boundary), and constants are left
    unchanged on every grid."""
    prob = _problem(4, (13, 9), (0, 1, 0, 1), EXT, 0.0, 0.0, t_final=0.1)
    prob.diffusion = lambda t, x, y: 0.002 * (1.0 + 0 * x + 0 * y)
    o = OracleSolver(prob)
    rng = np.random.Generator(np.random.PCG64(3))
    ks = _order_n_moments(o)
    before = {}
    for k in ks:
        if o.gx[k] == 1 and o.gy[k] == 1:
            o.u[k] = np.ascontiguousarray(rng.normal(size=o.u[k].shape))
        else:
            o.u[k] = np.full(o.u[k].shape, 3.5)
        before[k] = o.u[k].copy()
    o.diffuse(o.dt)
    assert any(o.gx[k] == 1 and o.gy[k] == 1 for k in ks)
    for k in ks:
        if o.gx[k] == 1 and o.gy[k] == 1:
            assert abs(o.u[k].sum() - before[k].sum()) < 1e-12
            assert not np.allclose(o.u[k], before[k])
        else:
            np.testing.assert_array_equal(o.u[k], before[k])


def test_zero_diffusion_is_plain_pn():
    prob = wl.line_source(N=5, n=30, s=0.1, t_final=0.2)
    a = OracleSolver(prob)
    a.run()
    prob.diffusion = _const(0.0)
    b = OracleSolver(prob)
    b.run()
    for x, y in zip(a.u, b.u):
        assert np.array_equal(x, y)


# ------------------------------------------------ extrapolation ghost rule
def test_extrapolation_ghosts_on_linear_fields():
    """Constant extrapolation onto ghost points (Sect. 4.2), pinned on linear
    fields by hand-computed differences.  P_1 on 6 x 5 cells of width h = 0.5,
    extrapolation on both axes, R_0^0 = 2 x + 3 y on G11 (cell centres):
      * D_x R_0^0 on the nodes 0..6 of G21: ghost cell 0 := cell 1 and ghost
        cell 7 := cell 6, so the difference is 0 at nodes 0 and 6 and exactly 2
        at the five inner nodes;
      * D_y R_0^0 on the nodes 0..5 of G12: 0 at nodes 0 and 5, exactly 3 inside.
    The odd residuals are W = -Mx(R_1^1, R_0^0) D_x R_0^0 and
    W = -My(I_1^1, R_0^0) D_y R_0^0 (their only couplings; the entries are the
    printed P_1 block, pinned in test_oracle_matrices).  A ghost taken one cell
    too far in (ghost := cell 2) would give -2 and -3 at the boundary nodes,
    an unassigned ghost (0) would give the boundary value itself.  Nodal
    fields need no ghost with extrapolation: R_1^1 = 5 x on G21 gives
    D_x = 5 in every cell, boundary cells included."""
    h = 0.5
    prob = _problem(1, (6, 5), (0, 6 * h, 0, 5 * h), EXT, 0.0, 0.0,
                    initial={0: lambda t, x, y: 2.0 * x + 3.0 * y,
                             1: lambda t, x, y: 5.0 * x + 0.0 * y})
    o = OracleSolver(prob)
    mx, my = float(o.Mx[1, 0]), float(o.My[2, 0])
    assert abs(mx - 1.0 / math.sqrt(3.0)) < 1e-15 and abs(abs(my) - 1.0 / math.sqrt(3.0)) < 1e-15
    W = o.flux(1)
    dx_expect = np.array([0.0, 2.0, 2.0, 2.0, 2.0, 2.0, 0.0])           # nodes 0..6
    dy_expect = np.array([0.0, 3.0, 3.0, 3.0, 3.0, 0.0])                # nodes 0..5
    assert W[1].shape == (5, 7) and W[2].shape == (6, 6)
    np.testing.assert_allclose(W[1], -mx * np.broadcast_to(dx_expect, (5, 7)), rtol=0, atol=1e-13)
    np.testing.assert_allclose(W[2], -my * np.broadcast_to(dy_expect[:, None], (6, 6)), rtol=0, atol=1e-13)
    # even residual from the nodal R_1^1 = 5 x (I_1^1 = 0): D_x = 5 on all 6 cells
    W0 = o.flux(0)
    np.testing.assert_allclose(W0[0], np.full((5, 6), -mx * 5.0), rtol=0, atol=1e-13)
