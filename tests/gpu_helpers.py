"""Shared helpers of the GPU tests: run a problem through the C-ABI and through
the oracle, and compare."""
import math

import numpy as np

import paper_1211_2205_amd as pa
from oracle.scheme import OracleSolver


def run_gpu(prob, nsteps=None, precision=None, variant=None, bind=True, init_arrays=None):
    s = pa.Solver.from_problem(prob, precision=precision)
    if init_arrays is not None:
        for k, a in enumerate(init_arrays):
            s.set_field_array(3, k, a)
    if bind:
        s.bind_torch()
    if variant is not None:
        s.set_variant(variant)
    n = s.nsteps if nsteps is None else nsteps
    s.advance(n)
    s.synchronize()
    out = s.moments()
    return s, out


def run_oracle(prob, nsteps=None, init_arrays=None, fused=False):
    o = OracleSolver(prob)
    if init_arrays is not None:
        for k, a in enumerate(init_arrays):
            o.u[k][:] = a
    n = o.nsteps if nsteps is None else nsteps
    o.advance(n, fused=fused)
    return o


def rel_l2(a_list, b_list):
    num = sum(float(np.sum((np.asarray(a) - np.asarray(b)) ** 2)) for a, b in zip(a_list, b_list))
    den = sum(float(np.sum(np.asarray(b) ** 2)) for b in b_list)
    return math.sqrt(num / den) if den > 0 else math.sqrt(num)


def max_rel(a_list, b_list):
    """max |a - b| over every moment and point, over max |b| (1 if b is zero)."""
    scale = max((float(np.max(np.abs(b))) for b in b_list if np.size(b)), default=0.0) or 1.0
    return max((float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) for a, b in zip(a_list, b_list) if np.size(b)),
               default=0.0) / scale


def moment_errors(a_list, b_list, floor=1e-2):
    """Per-moment relative L2 error: ||a_k - b_k|| / max(||b_k||, floor * max_j ||b_j||).
    The floor keeps moments that are zero (or nearly) by symmetry from
    dividing by their own round-off."""
    norms = [float(np.sqrt(np.sum(np.asarray(b, dtype=np.float64) ** 2))) for b in b_list]
    ref = floor * max(norms) if norms and max(norms) > 0 else 1.0
    out = []
    for a, b, nb in zip(a_list, b_list, norms):
        d = float(np.sqrt(np.sum((np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) ** 2)))
        out.append(d / max(nb, ref))
    return out


def assert_parity(a_list, b_list, tol, label="", moment_tol=None, elem_tol=None, floor=1e-2):
    """Parity of a device result a against the oracle b, moment by moment.

    Asserts three bounds:
      * relative L2 over all moments and points <= tol;
      * for every moment k, ||a_k - b_k|| / max(||b_k||, floor * max_j ||b_j||)
        <= moment_tol (default tol), so an error confined to one small moment
        cannot hide under the pooled norm;
      * max over all points of |a - b|, over max |b|, <= elem_tol (default
        tol), so an error confined to a few points (a boundary row) cannot
        either.
    Returns (pooled, worst moment error, its index, element error)."""
    assert len(a_list) == len(b_list)
    for a, b in zip(a_list, b_list):
        assert np.shape(a) == np.shape(b), (np.shape(a), np.shape(b))
    pooled = rel_l2(a_list, b_list)
    per = moment_errors(a_list, b_list, floor)
    k = int(np.argmax(per))
    elem = max_rel(a_list, b_list)
    mt = tol if moment_tol is None else moment_tol
    et = tol if elem_tol is None else elem_tol
    print(f"  {label} rel L2 {pooled:.3e}, worst moment {k}: {per[k]:.3e}, max element {elem:.3e}", flush=True)
    assert pooled <= tol, f"{label}: pooled relative L2 {pooled:.3e} > {tol:.1e}"
    assert per[k] <= mt, f"{label}: moment {k} relative L2 {per[k]:.3e} > {mt:.1e}"
    assert elem <= et, f"{label}: max element error {elem:.3e} > {et:.1e} of max |value|"
    return pooled, per[k], k, elem
