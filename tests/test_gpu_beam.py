"""Beam in void and medium (Sect. 6) on the GPU: sources on every moment from
the library's direction moments, void cells (zero decay), strong
Henyey-Greenstein scattering; against the oracle and the exact mass growth."""
import math

import numpy as np
import pytest

import paper_1211_2205_amd as pa
import workloads as wl
from gpu_helpers import assert_parity, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def test_beam_p9_150_matches_oracle():
    prob = wl.beam(N=9, n=150, t_final=0.6)
    s, g = run_gpu(prob)
    o = run_oracle(prob)
    assert_parity(g, o.u, 1e-12, f"beam P9 150^2 FP64 {s.nsteps} steps:")


def test_beam_p39_small_matches_oracle():
    # every one of the 820 moments carries a source; m ranges of several widths
    prob = wl.beam(N=39, n=60, t_final=0.2)
    s, g = run_gpu(prob, nsteps=20)
    o = run_oracle(prob, nsteps=20)
    assert_parity(g, o.u, 1e-12, "beam P39 60^2 FP64 20 steps:")


def test_beam_p39_150_fp32_mass_and_direction():
    """No absorption: the zeroth moment's mass grows by dt * sum(q_0) per step
    until radiation reaches the boundary; the beam moves along Omega_0."""
    prob = wl.beam(N=39, n=150, t_final=0.3, precision="fp32")
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    s.run()
    d = s.diagnostics()
    h = 1.2 / 150
    xc = -0.6 + (np.arange(150) + 0.5) * h
    X, Y = np.meshgrid(xc, xc)
    q0 = h * h * float(np.sum(prob.beam_profile(0.0, X, Y))) / math.sqrt(4 * math.pi)
    expect = s.nsteps * s.dt * q0
    print(f"beam P39 150^2 FP32: mass {d['mass']:.8f}, expected {expect:.8f}", flush=True)
    assert abs(d["mass"] - expect) < 1e-5 * expect
    r00 = s.get_moment(0)
    w = np.maximum(r00, 0.0)
    ang = math.atan2(float(np.sum(w * Y)), float(np.sum(w * X)))
    assert abs(ang - math.pi / 6) < 0.05, ang
