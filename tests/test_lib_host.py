"""Host-side checks of the native library (no GPU needed): every symbol the
header declares is exported, and the plan (moments, moment matrices, spectral
radius, time step) agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1211_2205_amd as pa
import workloads as wl
from oracle import pn
from oracle.scheme import OracleSolver

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "starmap.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(starmap_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(pa.LIB_PATH)
    names = _declared()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1211_2205_amd import _binding
    bound = {n for n, _, _ in _binding.SIGNATURES}
    assert set(_declared()) <= bound | {"starmap_field_fn"}


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9, 16, 31, 39])
def test_moment_matrices_match_oracle(N):
    Mx, My = pa.closure_pn(N)
    Ox, Oy = pn.real_matrices(N)
    np.testing.assert_allclose(Mx, Ox, rtol=0, atol=2e-15)
    np.testing.assert_allclose(My, Oy, rtol=0, atol=2e-15)


@pytest.mark.parametrize("N", [1, 3, 5, 7, 9, 31, 39, 60])
def test_moment_list_and_grids_match_oracle(N):
    mom = pn.moments(N)
    Ox, Oy = pn.real_matrices(N)
    gx, gy = pn.grid_classes(Ox, Oy)
    assert pa.num_moments(N) == len(mom)
    for k, (kind, l, m) in enumerate(mom):
        assert pa.moment_info(N, k) == (kind, l, m, gx[k], gy[k])


@pytest.mark.parametrize("N", list(range(1, 40)) + [60, 99])
def test_spectral_radius_is_largest_legendre_root(N):
    nodes, _ = np.polynomial.legendre.leggauss(N + 1)
    assert abs(pa.spectral_radius(N) - np.max(nodes)) < 1e-12


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_time_step_matches_oracle(name):
    prob = wl.config(name)
    s = pa.Solver.from_problem(prob)
    o_rho = pn.spectral_radius(pn.real_matrices(prob.N)[0])
    dx = (prob.ax[1] - prob.ax[0]) / prob.n[0]
    dt, n = pn.time_step(prob.cfl, dx, dx, o_rho, prob.t_final)
    t, sdt, done, total = s.time()
    assert total == n and sdt == dt and t == 0.0 and done == 0


def test_expected_step_counts():
    # line source P_3 100^2: 58 steps; checkerboard P_7 280^2: 246; P_39 1000^2: 666
    assert pa.Solver.from_problem(wl.config("c1")).nsteps == 58
    assert pa.Solver.from_problem(wl.config("c2")).nsteps == 246
    assert pa.Solver.from_problem(wl.config("c3")).nsteps == 666


def test_moment_shapes_follow_the_paper():
    s = pa.Solver(3, (7, 5), (0, 1, 0, 1), ("periodic", "extrapolation"))
    o = OracleSolver(wl.Problem("t", 3, (7, 5), (0, 1, 0, 1), ("periodic", "extrapolation"), 0.5, 1.0,
                                lambda t, x, y: 0 * x, lambda t, x, y: 0 * x))
    for k in range(10):
        nx, ny, x0, y0 = s.moment_shape(k)
        assert (ny, nx) == o.u[k].shape
        X, Y = o.grid.coords(o.gx[k], o.gy[k])
        assert abs(X[0, 0] - x0) < 1e-15 and abs(Y[0, 0] - y0) < 1e-15


def test_invalid_problems_are_rejected():
    with pytest.raises(pa.StarmapError):
        pa.Solver(0, (10, 10), (0, 1, 0, 1))
    with pytest.raises(pa.StarmapError):
        pa.Solver(3, (1, 10), (0, 1, 0, 1))
    with pytest.raises(pa.StarmapError):
        pa.Solver(3, (10, 10), (1, 0, 0, 1))
    with pytest.raises(pa.StarmapError):
        pa.Solver(3, (10, 10), (0, 1, 0, 1), cfl=-1.0)
    s = pa.Solver(3, (10, 10), (0, 1, 0, 1))
    with pytest.raises(pa.StarmapError):
        s.set_source(10, lambda t, x, y: x)
    assert s.workspace_bytes() > 10 * 11 * 11 * 8


def test_sweep_bytes_counts_every_plane():
    s = pa.Solver(39, (1000, 1000), (-1.5, 1.5, -1.5, 1.5), precision="fp32")
    b_odd = s.sweep_bytes(1)
    b_even = s.sweep_bytes(0)
    # odd sweep: 420 odd planes read+written, 400 even planes read (~1e6 points each)
    assert 4.0 * (2 * 420 + 400) * 1.0e6 < b_odd < 4.0 * (2 * 420 + 400 + 4) * 1.002e6
    assert 4.0 * (2 * 400 + 420) * 1.0e6 < b_even < 4.0 * (2 * 400 + 420 + 4) * 1.002e6


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 9, 10, 11, 15, 20, 31, 39, 60])
@pytest.mark.parametrize("tile", [(64, 4), (128, 2), (32, 8), (32, 16), (128, 4), (64, 8)])
def test_sweep_programs_are_consistent(N, tile):
    """Replay of the staged LDS window: every coupling of every row reads the
    plane the moment matrices name, for every m-range split."""
    from paper_1211_2205_amd import _binding as B
    L = pa.lib()
    for nchunks in sorted({1, 2, 3, 4, max(1, (N + 1) // 10), (N + 1) // 2 or 1}):
        rc = L.starmap_plan_check(N, tile[0], tile[1], nchunks)
        assert rc == 0, (N, tile, nchunks, L.starmap_last_error())


def test_separable_terms_are_validated_on_the_host():
    g = lambda x, y: x + 0 * y
    a = lambda t: 1.0 + t
    s = pa.Solver(3, (10, 10), (0, 1, 0, 1))
    base = s.workspace_bytes()
    for which, idx in (("absorption", 0), ("scattering", 0), ("scattering_order", 2), ("source", 1)):
        s.add_field_term(which, idx, g, a)
    # basis planes and the combination table take device memory
    assert s.workspace_bytes() > base
    L = pa._binding.lib()
    with pytest.raises(pa.StarmapError):
        pa._binding.check(L.starmap_add_field_term(s._h, 7, 0, pa._binding.FIELD_FN(), None,
                                                   pa._binding.TIME_FN(), None))
    with pytest.raises(pa.StarmapError):
        s.add_field_term("scattering_order", 0, g, a)   # orders are 1..N
    with pytest.raises(pa.StarmapError):
        s.add_field_term("scattering_order", 4, g, a)
    with pytest.raises(pa.StarmapError):
        s.add_field_term("source", 10, g, a)           # P_3 has 10 moments
    c = pa.Solver(5, (10, 10), (0, 1, 0, 1), closure="learned")
    with pytest.raises(pa.StarmapError):
        c.add_field_term("source", 20, g, a)           # order-5 moment of a closure solver


def test_separable_term_count_is_bounded():
    s = pa.Solver(3, (10, 10), (0, 1, 0, 1))
    g = lambda x, y: x + 0 * y
    for i in range(pa._binding.MAX_FIELD_TERMS):
        s.add_field_term("absorption", 0, g, (lambda i_: (lambda t: float(i_)))(i))
    before = s.workspace_bytes()
    with pytest.raises(pa.StarmapError):
        s.add_field_term("source", 0, g, lambda t: 1.0)
    # the rejected term left the plan unchanged
    assert s.workspace_bytes() == before


def test_header_constants_match_binding():
    txt = open(HEADER).read()
    defs = dict(re.findall(r"#define (STARMAP_[A-Z0-9_]+) (\d+)", txt))
    assert int(defs["STARMAP_FIELD_SCATTERING_ORDER"]) == pa._binding.FIELD_SCATTERING_ORDER
    assert int(defs["STARMAP_MAX_FIELD_TERMS"]) == pa._binding.MAX_FIELD_TERMS
    assert int(defs["STARMAP_FIELD_SOURCE"]) == pa._binding.FIELD_SOURCE


def test_tile_variants_are_enumerable():
    n = pa.variant_count()
    assert n >= 6
    s = pa.Solver(3, (40, 30), (0, 1, 0, 1))
    for v in range(n):
        s.set_variant(v)  # P_3 fits every tile within the 64 KiB assumed without a device
    with pytest.raises(pa.StarmapError, match="unknown variant"):
        s.set_variant(n)


def test_fpn_and_dn_settings_are_validated_on_the_host():
    s = pa.Solver(4, (12, 12), (0, 1, 0, 1))
    base = s.workspace_bytes()
    with pytest.raises(ValueError):
        s.set_filter_damping([0.0] * 4)
    with pytest.raises(pa.StarmapError):
        s.set_filter_damping([0.0, 1.0, -1.0, 0.0, 0.0])
    with pytest.raises(pa.StarmapError):
        s.set_filter_damping([0.0, 1.0, float("nan"), 0.0, 0.0])
    s.set_filter_damping(wl.filter_damping(4, 3.0))
    # per-order decay planes: more device memory
    assert s.workspace_bytes() > base
    s.set_filter_damping(None)
    d0 = s.workspace_bytes()
    s.set_diffusion(lambda t, x, y: 0.001 + 0 * x)
    # scratch and kappa planes for the N + 1 order-N moments
    assert s.workspace_bytes() > d0
    s.set_diffusion(None)
    assert s.workspace_bytes() == d0
    c = pa.Solver(5, (12, 12), (0, 1, 0, 1), closure="learned")
    with pytest.raises(pa.StarmapError):
        c.set_diffusion(lambda t, x, y: 0.001 + 0 * x)


def test_fused_mode_is_validated_on_the_host():
    # FP32: the tile fits the 64 KiB assumed without a device
    s = pa.Solver(5, (40, 30), (0, 1, 0, 1), precision="fp32")
    base = s.workspace_bytes()
    s.set_fused(True)
    # a second state buffer and the per-moment table
    assert s.workspace_bytes() > base + pa.num_moments(5) * 41 * 31 * 4
    s.set_fused(False)
    assert s.workspace_bytes() == base
    with pytest.raises(pa.StarmapError):
        pa.Solver(pa._binding.FUSED_MAX_ORDER + 1, (20, 20), (0, 1, 0, 1)).set_fused(True)
    with pytest.raises(pa.StarmapError):
        pa.Solver(5, (20, 20), (0, 1, 0, 1), closure="learned").set_fused(True)


@pytest.mark.parametrize("precision,n_ok,n_bad", [("fp64", 16000, 16400), ("fp32", 23000, 23200),
                                                  ("bf16", 23000, 23200)])
def test_create_rejects_planes_beyond_32bit_byte_offsets(precision, n_ok, n_bad):
    """The kernels address a plane with 32-bit byte offsets (element offset
    times the larger of the storage and compute sizes): starmap_create must
    reject a grid whose plane reaches 2^31 bytes and accept one just below.
    Host only: no such grid is ever launched."""
    def create(n):
        prob = wl.line_source(N=1, n=n, s=0.1, precision=precision)
        return pa.Solver.from_problem(prob)
    s = create(n_ok)
    s.close()
    with pytest.raises(pa.StarmapError) as e:
        create(n_bad)
    assert e.value.code == -1 and "32-bit" in str(e.value)


def test_range_width_setter():
    s = pa.Solver.from_problem(wl.config("c2"))
    assert s.chunk_width() == 8
    for w in (4, 6, 8):
        s.set_chunk_width(w)
        assert s.chunk_width() == w
    for bad in (0, 5, 12):
        with pytest.raises(pa.StarmapError):
            s.set_chunk_width(bad)
    assert s.chunk_width() == 8
