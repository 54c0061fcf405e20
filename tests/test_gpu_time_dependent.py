"""Time-dependent data on the device (Sect. 5.7): fields in time-separable form
sum a_i(t) g_i(x, y), whose decay and source planes are formed by the combine
kernel once per step, against the oracle, which samples the full fields at
t + dt/2 every step; and against the library's host re-sampling path."""
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
    for n in (splits or [s.nsteps]):
        s.advance(n)
        done += n
    s.advance(s.nsteps - done)
    s.synchronize()
    return s, s.moments()


def _host_path(prob):
    """The same problem with the separable form dropped: every field is a
    time-dependent callback re-sampled on the host each step."""
    import copy
    p = copy.copy(prob)
    p.separable = None
    return p


@pytest.mark.parametrize("n", [32, 45])
def test_manufactured_separable_fp64_matches_oracle(n):
    prob = wl.manufactured(n)
    s, g = _run(prob, splits=[3])
    o = run_oracle(prob)
    assert_parity(g, o.u, FP64_TOL, f"manufactured P3 {n}^2 separable on device, {s.nsteps} steps:")
    # the host re-sampling path gives the same answer
    _, h = _run(_host_path(prob))
    assert_parity(g, h, FP64_TOL, "device-combined vs host re-sampled data:")


@pytest.mark.parametrize("N,n", [(7, (40, 40)), (13, (33, 50))])
def test_pulsed_medium_fp64_matches_oracle(N, n):
    prob = wl.pulsed_medium(31 + N, N, n[0])
    prob.n = n
    s, g = _run(prob, splits=[1, 4])
    o = run_oracle(prob)
    err = assert_parity(g, o.u, FP64_TOL, f"pulsed medium P{N} {n}, {s.nsteps} steps:")[0]
    # the time dependence matters: data frozen at dt/2 give a far larger difference
    frozen = wl.pulsed_medium(31 + N, N, n[0])
    frozen.n = n
    frozen.time_dependent = False
    frozen.separable = None
    f = run_oracle(frozen)
    assert rel_l2(f.u, o.u) > 1e4 * max(err, 1e-16)


@pytest.mark.parametrize("precision,tol", [("fp32", FP32_TOL), ("bf16", 2e-2)])
def test_pulsed_medium_reduced_precision(precision, tol):
    prob = wl.pulsed_medium(40, 9, 48, precision=precision)
    _, g = _run(prob, precision=precision)
    o = run_oracle(prob)
    # bfloat16 rounds every stored value to 8 significant bits; a small
    # high-order moment inherits the rounding of its larger neighbours
    mt, et = (1e-1, 5e-2) if precision == "bf16" else (tol, tol)
    assert_parity(g, o.u, tol, f"pulsed medium P9 48^2 {precision}:", moment_tol=mt, elem_tol=et)


def test_separable_with_a_time_dependent_callback_uses_the_host_path():
    prob = wl.pulsed_medium(41, 5, 36)
    s = pa.Solver.from_problem(prob)
    # the source becomes a plain time-dependent callback (its terms are dropped)
    s.set_source(0, prob.source[0], time_dependent=1)
    s.bind_torch()
    s.run()
    g = s.moments()
    o = run_oracle(prob)
    assert_parity(g, o.u, FP64_TOL, "pulsed medium P5 36^2 with a callback source:")


def test_changing_a_constant_field_resamples_the_basis():
    prob = wl.manufactured(32)
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    s.advance(4)
    s.set_scattering(lambda t, x, y: 2.0 + 0 * x)
    s.advance(s.nsteps - 4)
    s.synchronize()
    from oracle.scheme import OracleSolver
    o = OracleSolver(prob)
    o.advance(4)
    o.prob.sigma_s0 = lambda t, x, y: np.full(np.broadcast(x, y).shape, 2.0)
    o.advance(o.nsteps - 4)
    assert_parity(s.moments(), o.u, FP64_TOL, "manufactured with scattering changed after 4 steps:")


def test_separable_errors():
    prob = wl.manufactured(16)
    s = pa.Solver.from_problem(prob)
    s.advance(1)
    with pytest.raises(pa.StarmapError):
        s.add_field_term("source", 2, lambda x, y: x, lambda t: 1.0)  # after the first device call
    with pytest.raises(pa.StarmapError):
        s.set_absorption(lambda t, x, y: x)  # a field given by terms is fixed now
    with pytest.raises(pa.StarmapError):
        pa.Batch([s])
    bad = pa.Solver(3, (16, 16), (0, 1, 0, 1))
    bad.add_field_term("absorption", 0, lambda x, y: 1.0 + 0 * x, lambda t: math.nan if t > 0.1 else 1.0)
    bad.advance(1)
    with pytest.raises(pa.StarmapError):
        bad.run()
