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
    scale = max(float(np.max(np.abs(b))) for b in b_list)
    return max(float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) for a, b in zip(a_list, b_list)) / scale
