"""HIP graphs in starmap_advance: the repeated sweep pairs replayed from
captured graphs give the same bits as the same launches made one by one, for
every run length (graphs of 16, 8, 4, 2 and 1 pairs), across several advance
calls with the program's own synchronising reads in between, after a tile
change (the graphs are rebuilt), with the D_N diffusion step and with the
learned closure inside the pairs."""
import numpy as np
import pytest

import paper_1211_2205_amd as pa
import workloads as wl
from oracle import closure as oc
from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pair(prob, closure_params=None):
    out = []
    for graphs in (True, False):
        kw = {"closure": "learned"} if closure_params is not None else {}
        s = pa.Solver.from_problem(prob, **kw)
        s.bind_torch()
        if closure_params is not None:
            s.load_closure(closure_params)
        s.set_graphs(graphs)
        out.append(s)
    return out


def _same(a, b, label):
    ga, gb = a.moments(), b.moments()
    for k, (x, y) in enumerate(zip(ga, gb)):
        assert np.array_equal(x, y), f"{label}: moment {k} differs"
    print(f"  {label}: identical", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replay_equals_eager_launches(precision):
    prob = wl.checkerboard(N=9, n=70, t_final=4.0, precision=precision)
    g, e = _pair(prob)
    assert g.nsteps > 70
    done = 0
    for n in (1, 2, 17, 33, 5, 16):   # every graph size, and remainders
        g.advance(n)
        e.advance(n)
        done += n
        _same(g, e, f"{precision} after {done} steps")
    # another tile: the captured graphs are dropped and rebuilt
    v0 = g.variant()[0]
    v1 = next(v for v in range(pa.variant_count()) if v != v0)
    for s in (g, e):
        s.set_variant(v1)
        s.set_chunk_width(6)
    g.advance(g.nsteps - done)
    e.advance(e.nsteps - done)
    _same(g, e, f"{precision} at t_final after a tile change")
    g.close()
    e.close()


def test_graph_replay_with_diffusion_step():
    prob = wl.line_source(N=7, n=61, s=0.1, t_final=0.8)
    h = (prob.ax[1] - prob.ax[0]) / prob.n[0]
    prob.diffusion = lambda t, x, y: 0.1 * h + 0 * x
    g, e = _pair(prob)
    for s in (g, e):
        s.advance(3)
        s.advance(s.nsteps - 3)
    _same(g, e, "D_N")


def test_graph_replay_with_learned_closure():
    prob = wl.random_medium(21, 5, 40)
    p = mlp.init(oc.N_IN, oc.N_HIDDEN, oc.N_OUT, 3, fan_in=oc.N_FEATURES)
    p["W3"] = p["W3"] * 0.2
    w = mlp.flatten({k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in p.items()})
    g, e = _pair(prob, closure_params=w)
    for s in (g, e):
        s.advance(2)
        s.advance(s.nsteps - 2)
    _same(g, e, "closure P_5")
