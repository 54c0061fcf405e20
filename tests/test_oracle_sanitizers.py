"""The oracle's C half-step code under AddressSanitizer and
UndefinedBehaviorSanitizer (host only): a driver built with both sanitizers
runs S^o S^e S^o on small grids of every boundary mix, including the smallest
grid (2 x 2) and ragged ones, and must finish without a report and give the
same values as the regular build of the oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as wl
from oracle.scheme import OracleSolver

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "oracle_sanitize_driver.c")

CASES = [
    (3, (2, 2), ("extrapolation", "extrapolation")),
    (3, (7, 5), ("periodic", "periodic")),
    (5, (6, 9), ("periodic", "extrapolation")),
    (4, (11, 3), ("extrapolation", "periodic")),
    (9, (13, 10), ("extrapolation", "extrapolation")),
]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp", "-o", exe, DRIVER, "-lm"]
    subprocess.check_call(cmd)
    return exe


@pytest.mark.parametrize("case", range(len(CASES)))
def test_oracle_half_steps_are_clean_under_sanitizers(driver, case):
    N, n, bc = CASES[case]
    prob = wl.Problem(name="asan", N=N, n=n, ax=(0.0, 1.0, 0.0, 1.0), bc=bc, cfl=0.5, t_final=0.1,
                      sigma_a=lambda t, x, y: 0 * x, sigma_s0=lambda t, x, y: 0 * x)
    o = OracleSolver(prob)
    init = wl.random_state(500 + case, [a.shape for a in o.u])
    lines = [f"{n[0]} {n[1]} {o.grid.px} {o.grid.py} {o.nmom}",
             " ".join(str(int(v)) for v in o.gx), " ".join(str(int(v)) for v in o.gy),
             " ".join(repr(float(v)) for v in o.Mx.ravel()), " ".join(repr(float(v)) for v in o.My.ravel())]
    for a in init:
        lines.append(" ".join(repr(float(v)) for v in np.asarray(a).ravel()))
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    got = np.array([float(v) for v in r.stdout.split()])
    # the same three half-steps in the regular build
    for k, a in enumerate(init):
        o.u[k][:] = a
    o._c = [np.full(a.shape, 1.0 + 0.1 * k) for k, a in enumerate(o.u)]
    o._q = [np.full(o.u[0].shape, 0.5)] + [None] * (o.nmom - 1)
    tau = 0.25 / n[0]
    o.half_step(1, tau)
    o.half_step(0, tau)
    o.emode = 1
    o.half_step(1, tau)
    want = np.concatenate([a.ravel() for a in o.u])
    assert got.shape == want.shape
    np.testing.assert_array_equal(got, want)
