"""Parity-fused passes (each step's odd and even half-steps in one pass over
the state, small orders) against the separate sweeps, bit for bit, and against
the oracle."""
import dataclasses

import numpy as np
import pytest

import paper_1211_2205_amd as pa
import workloads as wl
from gpu_helpers import assert_parity, rel_l2, run_oracle

pytestmark = pytest.mark.gpu

P, X = wl.BC_PERIODIC, wl.BC_EXTRAPOLATION


def _say(msg):
    print(msg, flush=True)


def _run(prob, fused, precision=None, splits=()):
    s = pa.Solver.from_problem(prob, precision=precision)
    if fused:
        s.set_fused(True)
    s.bind_torch()
    done = 0
    for n in splits:
        s.advance(n)
        done += n
    s.advance(s.nsteps - done)
    s.synchronize()
    out = s.moments()
    s.close()
    return out


def _identical(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


CASES = [
    ("checker5", lambda: wl.checkerboard(N=5, n=45, t_final=0.4), (45, 37), (X, X)),
    ("random7_periodic", lambda: wl.random_medium(51, 7, 40, t_final=0.2), (70, 33), (P, P)),
    ("random3_mixed", lambda: wl.random_medium(52, 3, 40, t_final=0.3), (33, 66), (P, X)),
    ("random1_mixed", lambda: wl.random_medium(53, 1, 40, t_final=0.3), (31, 29), (X, P)),
    ("line2", lambda: wl.line_source(N=2, n=50, s=0.1, half_width=1.0, t_final=0.3), (50, 50), (X, X)),
    # smaller than one 32 x 8 tile, and exactly one tile of points (nx + 1 = 32, ny + 1 = 8)
    ("tiny4_mixed", lambda: wl.random_medium(54, 4, 10, t_final=1.0), (7, 5), (X, P)),
    ("tile_edge6", lambda: wl.random_medium(55, 6, 10, t_final=0.2), (31, 7), (P, X)),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make,n,bc", CASES, ids=[c[0] for c in CASES])
def test_fused_equals_separate_sweeps_bitwise(name, make, n, bc, precision):
    prob = dataclasses.replace(make(), n=n, bc=bc, precision=precision)
    # the same split of the run into advance calls on both sides (two odd
    # half-steps at a call boundary equal one odd step only in exact arithmetic)
    a = _run(prob, False, precision, splits=(1, 2))
    b = _run(prob, True, precision, splits=(1, 2))
    _say(f"{name} {precision} {n} {bc}: identical {_identical(a, b)}, rel L2 {rel_l2(b, a):.3e}")
    assert _identical(a, b)
    if precision == "fp64":
        assert_parity(b, run_oracle(prob).u, 1e-12, f"{name} fused vs oracle:")


def test_fused_bf16_filtered_anisotropic():
    beam = dataclasses.replace(wl.beam(N=5, n=40, t_final=0.3), filter_damping=wl.filter_damping(5, 10.0))
    a = _run(beam, False)
    b = _run(beam, True)
    assert _identical(a, b)
    assert_parity(b, run_oracle(beam).u, 1e-12, "fused filtered beam vs oracle:")
    prob = wl.random_medium(54, 4, 48, t_final=0.2, precision="bf16")
    a = _run(prob, False, "bf16")
    b = _run(prob, True, "bf16")
    assert _identical(a, b)


def test_fused_errors_and_fallbacks():
    s = pa.Solver.from_problem(wl.random_medium(55, 3, 20, t_final=0.1))
    s.advance(1)
    with pytest.raises(pa.StarmapError):
        s.set_fused(True)  # after the first device call
    # a D_N solver keeps the separate sweeps (and their result)
    prob = wl.line_source(N=3, n=30, s=0.1, half_width=1.0, t_final=0.2)
    prob.diffusion = lambda t, x, y: 0.005 + 0 * x
    a = _run(prob, False)
    b = _run(prob, True)
    assert _identical(a, b)


def test_fused_lds_check_with_per_order_decay_planes():
    """FP64 P_7 with per-order decay planes (FP_N) needs 36 moment planes and
    16 decay planes of a 36 x 12 tile, 175.5 KB, more than a compute unit's
    LDS: refused whichever of the two calls comes first, before any launch."""
    _say("fused: FP64 P_7 FP_N LDS check")
    prob = wl.line_source(N=7, n=40, s=0.1, half_width=1.0, t_final=0.1, precision="fp64")
    damping = [0.0] + [0.1 * l for l in range(1, 8)]
    s = pa.Solver.from_problem(prob)
    s.set_fused(True)  # isotropic: 36 + 5 planes, 138 KB, fits
    s.set_filter_damping(damping)
    with pytest.raises(pa.StarmapError):
        s.advance(1)
    s.close()
    s = pa.Solver.from_problem(prob)
    s.set_filter_damping(damping)
    with pytest.raises(pa.StarmapError):
        s.set_fused(True)
    s.advance(1)  # still usable with the separate sweeps
    s.close()
