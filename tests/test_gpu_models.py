"""Moment models of the paper's outlook on the device against the oracle:
filtered P_N (per-order filter damping in the decay planes) and
diffusion-corrected P_N (a diffusion step on the order-N moments between the
two even half-steps)."""
import math

import numpy as np
import pytest

import paper_1211_2205_amd as pa
import workloads as wl
from gpu_helpers import assert_parity, rel_l2, run_oracle

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def _run(prob, precision=None, splits=None):
    s = pa.Solver.from_problem(prob, precision=precision)
    s.bind_torch()
    done = 0
    for n in (splits or []):
        s.advance(n)
        done += n
    s.advance(s.nsteps - done)
    s.synchronize()
    return s, s.moments()


def _fpn_checker(N=7, n=70, precision="fp64"):
    prob = wl.checkerboard(N=N, n=n, t_final=0.6, precision=precision)
    prob.filter_damping = wl.filter_damping(N, 8.0, power=4)
    return prob


@pytest.mark.parametrize("N", [5, 8])
def test_fpn_fp64_matches_oracle(N):
    prob = _fpn_checker(N)
    s, g = _run(prob, splits=[2])
    o = run_oracle(prob)
    err = assert_parity(g, o.u, FP64_TOL, f"FP_N checkerboard P{N} 70^2:")[0]
    # the damping matters
    plain = _fpn_checker(N)
    plain.filter_damping = None
    assert rel_l2(run_oracle(plain).u, o.u) > 1e6 * max(err, 1e-17)


def test_fpn_fp32_and_anisotropic_beam():
    prob = _fpn_checker(7, precision="fp32")
    _, g = _run(prob, precision="fp32")
    assert_parity(g, run_oracle(prob).u, FP32_TOL, "FP_N checkerboard P7 fp32:")
    beam = wl.beam(N=9, n=60, t_final=0.3)
    beam.filter_damping = wl.filter_damping(9, 20.0, power=2)
    _, g = _run(beam)
    assert_parity(g, run_oracle(beam).u, FP64_TOL, "FP_N beam P9 60^2 (anisotropic scattering):")


def test_fpn_with_separable_data_and_a_later_change():
    """Damping constants enter the device combination of time-separable decay
    planes; changing the damping mid-run is picked up by both paths."""
    prob = wl.manufactured(32)
    prob.filter_damping = wl.filter_damping(3, 4.0, power=1)
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    s.advance(5)
    d2 = wl.filter_damping(3, 9.0, power=2)
    s.set_filter_damping(d2)
    s.advance(s.nsteps - 5)
    s.synchronize()
    from oracle.scheme import OracleSolver
    o = OracleSolver(prob)
    o.advance(5)
    o.prob.filter_damping = d2
    o.advance(o.nsteps - 5)
    assert_parity(s.moments(), o.u, FP64_TOL, "FP_N manufactured, damping changed after 5 steps:")


def _dn_problem(N, n, bc, precision="fp64"):
    prob = wl.line_source(N=N, n=n, s=0.08, half_width=1.0, t_final=0.4, precision=precision)
    prob.bc = bc
    h = 2.0 / n
    prob.diffusion = lambda t, x, y: 0.12 * h * (1.0 + 0.5 * np.sin(math.pi * x) * np.cos(0.5 * math.pi * y))
    return prob


@pytest.mark.parametrize("N,bc", [(4, (wl.BC_EXTRAPOLATION, wl.BC_EXTRAPOLATION)),
                                  (5, (wl.BC_PERIODIC, wl.BC_EXTRAPOLATION)),
                                  (9, (wl.BC_PERIODIC, wl.BC_PERIODIC))])
def test_dn_fp64_matches_oracle(N, bc):
    prob = _dn_problem(N, 61, bc)
    s, g = _run(prob, splits=[1, 3])
    o = run_oracle(prob)
    err = assert_parity(g, o.u, FP64_TOL, f"D_N line source P{N} 61^2 {bc}: {s.nsteps} steps,")[0]
    plain = _dn_problem(N, 61, bc)
    plain.diffusion = None
    assert rel_l2(run_oracle(plain).u, o.u) > 1e4 * max(err, 1e-17)


def test_dn_fp32_and_separable():
    prob = _dn_problem(7, 64, (wl.BC_EXTRAPOLATION, wl.BC_EXTRAPOLATION), precision="fp32")
    _, g = _run(prob, precision="fp32")
    assert_parity(g, run_oracle(prob).u, FP32_TOL, "D_N line source P7 fp32:")
    man = wl.manufactured(40)
    man.diffusion = lambda t, x, y: 1e-4 + 0 * x
    _, g = _run(man)
    assert_parity(g, run_oracle(man).u, FP64_TOL, "D_N manufactured (separable data):")


def test_dn_errors():
    prob = _dn_problem(4, 40, (wl.BC_EXTRAPOLATION, wl.BC_EXTRAPOLATION))
    prob.diffusion = lambda t, x, y: 10.0 + 0 * x   # far beyond the explicit limit
    s = pa.Solver.from_problem(prob)
    with pytest.raises(pa.StarmapError, match="unstable"):
        s.advance(1)
    ok = pa.Solver.from_problem(_dn_problem(4, 40, (wl.BC_EXTRAPOLATION, wl.BC_EXTRAPOLATION)))
    ok.advance(1)
    with pytest.raises(pa.StarmapError):
        ok.set_diffusion(lambda t, x, y: 0 * x)  # after the first device call
    with pytest.raises(pa.StarmapError):
        pa.Batch([ok])
