"""starmap_diagnostics_noalloc (partials in the library's static device
scratch, no allocation) against starmap_diagnostics (partials in the solver's
workspace): the same four results, on two calls in a row, the second on a
smaller problem, each checked straight through the C ABI."""
import ctypes

import numpy as np
import pytest

import paper_1211_2205_amd as pa
import workloads as wl
from paper_1211_2205_amd import _binding as B

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _diag(fn, s):
    m, l2, mx = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    nf = ctypes.c_int32()
    rc = fn(s._h, ctypes.byref(m), ctypes.byref(l2), ctypes.byref(mx), ctypes.byref(nf))
    return rc, (m.value, l2.value, mx.value, nf.value)


def _check(prob, steps):
    L = B.lib()
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    s.advance(steps)
    s.synchronize()
    rc0, ref = _diag(L.starmap_diagnostics, s)
    rc1, got = _diag(L.starmap_diagnostics_noalloc, s)
    print(f"{prob.name} {prob.n}: workspace {ref}, static scratch {got}", flush=True)
    assert rc0 == 0 and rc1 == 0
    assert got[3] == ref[3] == 0
    for a, b in zip(got[:3], ref[:3]):
        assert abs(a - b) <= 1e-12 * abs(b)
    s.close()
    return got


def test_noalloc_diagnostics_equal_workspace_diagnostics():
    big = wl.config("c2")                     # P_7, 280^2: 36 planes x 5 blocks
    big.n = (280, 280)
    small = wl.line_source(N=3, n=40, s=0.1)  # P_3, 40^2: 10 planes x 1 block
    a = _check(big, 12)
    b = _check(small, 5)
    assert a != b


def test_noalloc_diagnostics_errors():
    L = B.lib()
    s = pa.Solver.from_problem(wl.line_source(N=3, n=16, s=0.1))
    rc, _ = _diag(L.starmap_diagnostics_noalloc, s)  # no device state yet: it would allocate
    assert rc == -5
    # too many reduction blocks for the static scratch: P_60 (1891 planes) on
    # 2201 rows needs 1891 x 35 > 65536 blocks
    prob = wl.line_source(N=60, n=2, s=0.1, precision="bf16")
    prob.n = (2, 2200)
    big = pa.Solver.from_problem(prob)
    assert big.nmom * ((2200 + 1 + 63) // 64) > 65536
    big.bind_torch()
    big.diagnostics()  # the workspace variant sets the device state up
    rc, _ = _diag(L.starmap_diagnostics_noalloc, big)
    assert rc == -1 and b"static scratch" in L.starmap_last_error()
    s.close()
    big.close()
