"""GPU parity: the HIP path (through the C-ABI) against the oracle on the same
seeded inputs.  FP64 must agree to 1e-12 relative L2 over all moments and
points; FP32 storage to 1e-5; BF16 storage is reported against a loose bound."""
import math
import sys

import numpy as np
import pytest

import paper_1211_2205_amd as pa
import workloads as wl
from gpu_helpers import assert_parity, rel_l2, run_gpu, run_oracle
from oracle.scheme import OracleSolver

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _const(v):
    return lambda t, x, y: np.full(np.broadcast(x, y).shape, float(v))


def _random_init(prob, seed):
    o = OracleSolver(prob)
    return wl.random_state(seed, [a.shape for a in o.u])


# ------------------------------------------------------------ small cases
SMALL = [
    # N, (nx, ny), bc, anisotropic, source
    (1, (9, 7), ("periodic", "periodic"), False, False),
    (3, (37, 23), ("extrapolation", "extrapolation"), False, True),
    (3, (37, 23), ("periodic", "extrapolation"), True, True),
    (4, (30, 41), ("extrapolation", "periodic"), False, True),
    (5, (2, 2), ("extrapolation", "extrapolation"), False, False),
    (5, (3, 5), ("periodic", "periodic"), True, False),
    (7, (70, 9), ("extrapolation", "extrapolation"), True, True),
    (9, (65, 66), ("periodic", "periodic"), False, True),
    (15, (20, 33), ("extrapolation", "extrapolation"), False, False),
    (39, (17, 12), ("extrapolation", "periodic"), False, True),
    (2, (2, 2), ("periodic", "periodic"), True, True),
    (2, (5, 2), ("extrapolation", "periodic"), False, True),
]


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_small_cases_fp64(case):
    N, n, bc, aniso, src = SMALL[case]
    _say(f"small case {case}: N={N} n={n} bc={bc} aniso={aniso} src={src}")
    rng = np.random.default_rng(case)
    sa = rng.uniform(0, 2, size=4)
    prob = wl.Problem(
        name="small", N=N, n=n, ax=(-0.3, 0.9, 0.1, 1.3), bc=bc, cfl=0.5, t_final=0.4,
        sigma_a=lambda t, x, y: sa[0] + sa[1] * np.sin(3 * x) * np.cos(2 * y),
        sigma_s0=lambda t, x, y: sa[2] + 0 * x,
        sigma_sl=(lambda l, t, x, y: 0.8 ** l * (1 + 0 * x)) if aniso else None,
        source={0: lambda t, x, y: np.exp(-x * x - y * y)} if src else {})
    init = _random_init(prob, 100 + case)
    nsteps = 7
    _, g = run_gpu(prob, nsteps=nsteps, init_arrays=init)
    o = run_oracle(prob, nsteps=nsteps, init_arrays=init)
    assert_parity(g, o.u, FP64_TOL, f"small case {case}")


def test_c1_line_source_fp64_full_run():
    prob = wl.config("c1")
    s, g = run_gpu(prob)
    o = run_oracle(prob)
    assert s.nsteps == 58
    assert_parity(g, o.u, FP64_TOL, f"C1 P3 100^2 FP64, {s.nsteps} steps:")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_step_and_step_splits(precision):
    """The degenerate step counts of the composition: a run of one step
    (S^o_{dt/2} S^e_dt S^o_{dt/2}, three sweeps), advance(0) as a no-op, and one
    run advanced in uneven pieces (1, 2, 5, 16, 3 steps: graphs of 16/8/4/2/1
    sweep pairs and their remainders; every piece closes with an odd half-step
    and the next opens with one, where one advance merges them into a full odd
    step: equal in exact arithmetic) against one advance over all steps and
    the oracle."""
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    prob = wl.random_medium(61, 5, 37, t_final=0.8, precision=precision)
    prob.n = (37, 29)
    prob.bc = (wl.BC_PERIODIC, wl.BC_EXTRAPOLATION)
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    assert s.nsteps >= 27
    init = [m.copy() for m in s.moments()]
    s.advance(0)
    assert s.time()[2] == 0
    assert all(np.array_equal(a, b) for a, b in zip(s.moments(), init))
    s.advance(1)
    assert s.time()[2] == 1
    assert_parity(s.moments(), run_oracle(prob, nsteps=1).u, tol, f"{precision} one step")
    for k in (2, 5, 16, 3):
        s.advance(k)
    pieces = s.moments()
    assert s.time()[2] == 27
    s.reset()
    s.advance(27)
    whole = s.moments()
    assert_parity(pieces, whole, tol, f"{precision} pieces against one advance")
    o = run_oracle(prob, nsteps=27).u
    assert_parity(whole, o, tol, f"{precision} 27 steps")
    assert_parity(pieces, o, tol, f"{precision} 27 steps in pieces")
    s.close()


def test_maximum_order_p99():
    """The largest moment order the library accepts, N = 99 (5050 moments, 17
    m ranges of the default width), on a ragged 20 x 13 grid with an
    extrapolation and a periodic axis: the whole run (5 steps) against the
    oracle, FP64."""
    prob = wl.random_medium(71, 99, 20, t_final=0.25, precision="fp64")
    prob.n = (20, 13)
    prob.bc = (wl.BC_EXTRAPOLATION, wl.BC_PERIODIC)
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    assert s.nsteps == 5
    s.run()
    assert_parity(s.moments(), run_oracle(prob).u, FP64_TOL, "P_99 20x13, 5 steps")
    s.close()


@pytest.mark.parametrize("N", [5, 13, 39])
def test_tile_variants_are_bitwise_identical(N, monkeypatch):
    """Every compiled tile variant and every split of the moments into m
    ranges gives the same bits: the arithmetic per point does not depend on
    the tiling."""
    prob = wl.checkerboard(N=N, n=77, t_final=0.5)
    ref = None
    for width in (2, 5, 8, 12):
        monkeypatch.setenv("STARMAP_CHUNK_WIDTH", str(width))
        for v in range(pa.variant_count()):
            s = pa.Solver.from_problem(prob)
            s.bind_torch()
            try:
                s.set_variant(v)
            except pa.StarmapError:
                continue
            s.advance(9)
            out = s.moments()
            if ref is None:
                ref = out
            else:
                for a, b in zip(out, ref):
                    assert np.array_equal(a, b), f"variant {v} width {width} differs"
    assert ref is not None


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_tile_orders_are_bitwise_identical(precision, monkeypatch):
    """Row strips, column strips and row-by-row numbering of the tiles (the
    order workgroups take them in) give the same bits, on a ragged grid whose
    tile rows and columns do not divide into the strips."""
    prob = wl.random_medium(33, 9, 150, t_final=0.2, precision=precision)
    prob.n = (150, 77)
    prob.bc = (wl.BC_PERIODIC, wl.BC_EXTRAPOLATION)
    ref = None
    for strip in ("8", "1", "3", "-2", "-5", "-8"):
        monkeypatch.setenv("STARMAP_TILE_STRIP", strip)
        s = pa.Solver.from_problem(prob, precision=precision)
        s.bind_torch()
        s.advance(6)
        out = s.moments()
        s.close()
        if ref is None:
            ref = out
        else:
            for a, b in zip(out, ref):
                assert np.array_equal(a, b), f"strip {strip} differs"


@pytest.mark.parametrize("case", ["checker13", "mixed9", "periodic39"])
def test_fp32_tile_variants_are_bitwise_identical(case, monkeypatch):
    """FP32 storage: every tile variant and several m-range widths give the
    same bits, on extrapolated, periodic and mixed boundaries with ragged
    grids; and match the oracle."""
    if case == "checker13":
        prob = wl.checkerboard(N=13, n=77, t_final=0.5, precision="fp32")
    elif case == "mixed9":
        prob = wl.random_medium(31, 9, 70, t_final=0.3, precision="fp32")
        prob.n = (70, 45)
        prob.bc = (wl.BC_PERIODIC, wl.BC_EXTRAPOLATION)
    else:
        prob = wl.random_medium(32, 39, 40, t_final=0.2, precision="fp32")
        prob.n = (67, 40)
        prob.bc = (wl.BC_PERIODIC, wl.BC_PERIODIC)
    ref, tried = None, []
    for width in (4, 8):
        monkeypatch.setenv("STARMAP_CHUNK_WIDTH", str(width))
        for v in range(pa.variant_count()):
            s = pa.Solver.from_problem(prob)
            s.bind_torch()
            try:
                s.set_variant(v)
            except pa.StarmapError:
                continue
            _say(f"  {case} variant {v} width {width}")
            tried.append((v, width))
            s.advance(7)
            out = s.moments()
            if ref is None:
                ref = out
            else:
                for a, b in zip(out, ref):
                    assert np.array_equal(a, b), f"variant {v} width {width} differs"
    assert len(tried) >= 8
    o = run_oracle(prob, nsteps=7)
    assert_parity(ref, o.u, FP32_TOL, f"{case} FP32 vs oracle:")


@pytest.mark.parametrize("bc", [("extrapolation", "extrapolation"), ("periodic", "periodic"),
                                ("periodic", "extrapolation")])
def test_bf16_tile_variants_are_bitwise_identical(bc, monkeypatch):
    """BF16 storage: tiles of 512 points move x-adjacent pairs as one 32-bit
    access away from the grid's right edge (and single values at the edge);
    tiles of 256 points move single values.  Every variant gives the same
    bits, on a grid (150 x 77) that has both kinds of 512-point tiles."""
    prob = wl.random_medium(35, 9, 150, t_final=0.2, precision="bf16")
    prob.n = (150, 77)
    prob.bc = bc
    ref, tried = None, []
    for width in (4, 8):
        monkeypatch.setenv("STARMAP_CHUNK_WIDTH", str(width))
        for v in range(pa.variant_count()):
            s = pa.Solver.from_problem(prob, precision="bf16")
            s.bind_torch()
            try:
                s.set_variant(v)
            except pa.StarmapError:
                continue
            tried.append((v, width))
            s.advance(6)
            out = s.moments()
            if ref is None:
                ref = out
            else:
                for a, b in zip(out, ref):
                    assert np.array_equal(a, b), f"variant {v} width {width} differs"
    assert len(tried) >= 8
    o = run_oracle(prob, nsteps=6)
    assert_parity(ref, o.u, 2e-2, f"BF16 {bc} vs oracle:", moment_tol=1e-1, elem_tol=5e-2)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("bc", [("periodic", "periodic"), ("extrapolation", "periodic")])
def test_grid_of_whole_tiles_variants_are_bitwise_identical(precision, bc, monkeypatch):
    """A 128 x 64 grid holds whole tiles of every variant, so every tile takes
    the pair and wide paths (no right-edge tile with single accesses) and the
    halo of the last tile column wraps or clamps at the grid's edge.  Every
    variant gives the same bits, and the result matches the oracle."""
    prob = wl.random_medium(36, 9, 128, t_final=0.2, precision=precision)
    prob.n = (128, 64)
    prob.bc = bc
    ref, tried = None, []
    for width in (4, 6):
        monkeypatch.setenv("STARMAP_CHUNK_WIDTH", str(width))
        for v in range(pa.variant_count()):
            s = pa.Solver.from_problem(prob, precision=precision)
            s.bind_torch()
            try:
                s.set_variant(v)
            except pa.StarmapError:
                continue
            tried.append((v, width))
            s.advance(6)
            out = s.moments()
            s.close()
            if ref is None:
                ref = out
            else:
                for a, b in zip(out, ref):
                    assert np.array_equal(a, b), f"variant {v} width {width} differs"
    assert len(tried) >= 8
    o = run_oracle(prob, nsteps=6)
    if precision == "fp32":
        assert_parity(ref, o.u, FP32_TOL, f"FP32 {bc} 128x64 vs oracle:")
    else:
        assert_parity(ref, o.u, 2e-2, f"BF16 {bc} 128x64 vs oracle:", moment_tol=1e-1, elem_tol=5e-2)


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_c2_checkerboard_full_run(precision, tol):
    prob = wl.config("c2")
    s, g = run_gpu(prob, precision=precision)
    o = run_oracle(prob)
    assert s.nsteps == 246
    assert_parity(g, o.u, tol, f"C2 P7 280^2 {precision}, {s.nsteps} steps:")


def test_bf16_storage_error_is_bounded():
    prob = wl.config("c1")
    _, g = run_gpu(prob, precision="bf16")
    o = run_oracle(prob)
    # bfloat16 keeps 8 significant bits (relative rounding 2^-9 per store); a
    # small high-order moment inherits the rounding of its larger neighbours
    assert_parity(g, o.u, 2e-2, "C1 BF16 storage:", moment_tol=1e-1, elem_tol=5e-2)


def test_time_dependent_manufactured_problem_fp64():
    """MMS setting of the paper (time-dependent absorption and source,
    anisotropic scattering, periodic) on the device vs the oracle."""
    m = math.sqrt(2.0) * math.sqrt(2.0 / 3.0) / 2.0
    exact = lambda t, x, y: math.exp(-t) * np.sin(2 * math.pi * x) ** 2 + 0 * y
    prob = wl.Problem(
        name="mms", N=3, n=(32, 32), ax=(0, 1, 0, 1), bc=("periodic", "periodic"), cfl=0.5, t_final=0.5,
        sigma_a=lambda t, x, y: t * np.cos(2 * math.pi * y) + 0 * x, sigma_s0=_const(1.0),
        sigma_sl=lambda l, t, x, y: 0.9 ** l + 0 * x,
        source={0: lambda t, x, y: exact(t, x, y) * (t * np.cos(2 * math.pi * y) - 1.0),
                1: lambda t, x, y: m * 2 * math.pi * math.exp(-t) * np.sin(4 * math.pi * x) + 0 * y},
        initial={0: exact}, time_dependent=True)
    _, g = run_gpu(prob)
    o = run_oracle(prob)
    assert_parity(g, o.u, FP64_TOL, "MMS P3 32^2 time-dependent:")


# -------------------------------------------- full-size large line source
C3_CENTERS = [(0.0, 0.0), (-1.45, -1.45), (1.45, 1.45), (-1.45, 1.45), (1.45, -1.45), (0.0, -1.47), (1.47, 0.3)]


def _window_problem(prob, i0, j0, w):
    h = (prob.ax[1] - prob.ax[0]) / prob.n[0]
    sub = wl.Problem(name="win", N=prob.N, n=(w, w),
                     ax=(prob.ax[0] + i0 * h, prob.ax[0] + (i0 + w) * h, prob.ax[2] + j0 * h, prob.ax[2] + (j0 + w) * h),
                     bc=prob.bc, cfl=prob.cfl, t_final=prob.t_final, sigma_a=prob.sigma_a, sigma_s0=prob.sigma_s0,
                     source=prob.source, initial=prob.initial)
    return sub


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_c3_full_size_windows(precision, tol):
    """Large line source at its full size (P_39, 1000^2) in the benchmark's
    launch configuration, Gaussians at the centre, corners and edges.  After K
    steps a point depends only on points within 2K+1 cells, so the oracle run
    on a window reproduces the window's interior exactly; windows that touch
    the true boundary check the boundary handling."""
    K = 3
    prob = wl.line_source_multi(N=39, n=1000, s=0.01, centers=C3_CENTERS, precision=precision)
    _say(f"C3 windows {precision}: GPU run of {K} steps")
    s = pa.Solver.from_problem(prob, precision=precision)
    s.bind_torch()
    s.autotune(2)
    _say(f"  variant {s.variant()}")
    s.advance(K)
    s.synchronize()
    assert s.dt == pytest.approx(1.0 / 666, rel=1e-15)
    g = s.moments()
    w, margin = 40, 2 * K + 2
    n = prob.n[0]
    windows = [(480, 480), (0, 0), (n - w, n - w), (0, n - w), (n - w, 0), (480, 0), (n - w, 590)]
    worst = 0.0
    for (i0, j0) in windows:
        sub = _window_problem(prob, i0, j0, w)
        o = run_oracle(sub, nsteps=K)
        ga, oa = [], []
        for k in range(o.nmom):
            ny_k, nx_k = o.u[k].shape
            gk = g[k][j0:j0 + ny_k, i0:i0 + nx_k]
            lo_x = 0 if i0 == 0 else margin
            lo_y = 0 if j0 == 0 else margin
            hi_x = nx_k if i0 + w == n else nx_k - margin
            hi_y = ny_k if j0 + w == n else ny_k - margin
            ga.append(gk[lo_y:hi_y, lo_x:hi_x])
            oa.append(o.u[k][lo_y:hi_y, lo_x:hi_x])
        err, _, _, _ = assert_parity(ga, oa, tol, f"window ({i0},{j0}):")
        worst = max(worst, err)
    assert worst < tol


def test_c3_full_run_invariants_fp64():
    """Full P_39 1000^2 run to t = 1 in FP64: the front (speed < 1) never
    reaches the boundary, so the zeroth-moment mass stays at its initial value
    to round-off; R00 stays symmetric under x <-> y and under the mirrors."""
    prob = wl.config("c3", precision="fp64")
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    s.autotune(2)
    d0 = s.diagnostics()
    s.run()
    d1 = s.diagnostics()
    _say(f"C3 FP64 full run: mass {d0['mass']:.15f} -> {d1['mass']:.15f}, l2 {d0['l2']:.6e} -> {d1['l2']:.6e}")
    assert abs(d1["mass"] - d0["mass"]) < 1e-12 * abs(d0["mass"])
    r = s.get_moment(0)
    sc = np.max(np.abs(r))
    assert np.max(np.abs(r - r.T)) < 1e-12 * sc
    assert np.max(np.abs(r - r[::-1, :])) < 1e-12 * sc
    assert np.max(np.abs(r - r[:, ::-1])) < 1e-12 * sc


def test_c3_fp32_full_run_against_fp64():
    """Large line source (P_39, 1000^2) to t_final = 1 (666 steps) with FP32
    storage against the same run with FP64 storage, both on the device in the
    benchmark's launch configuration (autotuned tile).  The FP64 run stands in
    for the oracle at this size (it matches the oracle to 1e-12 on the
    full-size windows above and on the C1/C2 full runs); the comparison is
    plane by plane: relative L2 over all moments <= 1e-5, every moment's
    relative L2 (floor: 1% of the largest moment norm) <= 1e-5, and the
    largest pointwise error <= 1e-5 of max |u|."""
    prob64 = wl.config("c3", precision="fp64")
    prob32 = wl.config("c3", precision="fp32")
    runs = {}
    for name, prob in (("fp64", prob64), ("fp32", prob32)):
        s = pa.Solver.from_problem(prob)
        s.bind_torch()
        s.autotune(2)
        _say(f"C3 {name}: variant {s.variant()}, {s.nsteps} steps")
        s.run()
        assert s.time()[2] == 666
        runs[name] = s
    a, b = runs["fp32"], runs["fp64"]
    num = den = 0.0
    worst_k, worst_m, elem, scale = -1, 0.0, 0.0, 0.0
    norms, errs = [], []
    for k in range(b.nmom):
        gb = b.get_moment(k)
        ga = a.get_moment(k)
        d = ga - gb
        e2, n2 = float(np.sum(d * d)), float(np.sum(gb * gb))
        num += e2
        den += n2
        norms.append(math.sqrt(n2))
        errs.append(math.sqrt(e2))
        elem = max(elem, float(np.max(np.abs(d))))
        scale = max(scale, float(np.max(np.abs(gb))))
    floor = 1e-2 * max(norms)
    per = [e / max(n, floor) for e, n in zip(errs, norms)]
    worst_k = int(np.argmax(per))
    worst_m = per[worst_k]
    pooled = math.sqrt(num / den)
    _say(f"C3 FP32 vs FP64 at t_final: rel L2 {pooled:.3e}, worst moment {worst_k}: {worst_m:.3e}, "
         f"max element {elem / scale:.3e}")
    assert pooled <= FP32_TOL
    assert worst_m <= FP32_TOL
    assert elem <= FP32_TOL * scale
    for s in runs.values():
        s.close()


# ---------------------------------------------------- runtime behaviour
def test_checkpoint_resume_is_bitwise():
    prob = wl.config("c2")
    prob.n = (70, 70)
    a = pa.Solver.from_problem(prob)
    a.bind_torch()
    a.advance(5)
    a.advance(6)
    ref = a.moments()
    b = pa.Solver.from_problem(prob)
    b.bind_torch()
    b.advance(5)
    buf, t, st = b.get_state()
    c = pa.Solver.from_problem(prob)
    c.bind_torch()
    c.set_state(buf, t, st)
    c.advance(6)
    assert c.time()[2] == 11
    for x, y in zip(c.moments(), ref):
        assert np.array_equal(x, y)


def test_library_allocation_equals_torch_binding():
    prob = wl.line_source(N=3, n=64, s=0.1)
    _, a = run_gpu(prob, nsteps=10, bind=True)
    _, b = run_gpu(prob, nsteps=10, bind=False)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_diagnostics_match_oracle():
    prob = wl.config("c2")
    prob.n = (56, 56)
    s, g = run_gpu(prob, nsteps=20)
    o = run_oracle(prob, nsteps=20)
    d = s.diagnostics()
    assert d["nonfinite"] == 0
    assert abs(d["mass"] - o.mass()) < 1e-12 * abs(o.mass())
    assert abs(d["l2"] - o.l2()) < 1e-12 * o.l2()
    assert d["maxabs"] == pytest.approx(max(float(np.max(np.abs(a))) for a in o.u), rel=1e-12)


def test_nonfinite_state_is_reported():
    prob = wl.line_source(N=3, n=32, s=0.1)
    prob.initial = {0: lambda t, x, y: np.where((x > 0.5) & (y > 0.5), np.nan, 1.0)}
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    s.advance(2)
    with pytest.raises(pa.StarmapError) as e:
        s.diagnostics()
    assert e.value.code == -4
    d = s.diagnostics(raise_unstable=False)
    assert d["nonfinite"] > 0


def test_unstable_cfl_blows_up_on_device():
    """cfl beyond 1/sqrt2 amplifies the checkerboard mode (same as the oracle)."""
    prob = wl.Problem(name="cfl", N=3, n=(32, 32), ax=(0, 1, 0, 1), bc=("periodic", "periodic"), cfl=0.72,
                      t_final=60 * 0.72 / 32 / pa.spectral_radius(3), sigma_a=_const(0), sigma_s0=_const(0))
    init = _random_init(prob, 7)
    s, g = run_gpu(prob, init_arrays=init)
    o = run_oracle(prob, init_arrays=init)
    assert s.diagnostics()["l2"] > 1e3 * math.sqrt(sum(float(np.sum(a * a)) for a in init) / 32 / 32)
    assert rel_l2(g, o.u) < 1e-9
