"""Batched heterogeneous solves on the GPU: one launch per sweep over all
instances still running, the whole run in one HIP graph.  Every instance of a
batch must equal its own single-instance run bit for bit (same tile, same
programs, same arithmetic) and the oracle within the parity tolerance."""
import dataclasses

import numpy as np
import pytest

import paper_1211_2205_amd as pa
import workloads as wl
from gpu_helpers import assert_parity, run_oracle

pytestmark = pytest.mark.gpu

P, X = wl.BC_PERIODIC, wl.BC_EXTRAPOLATION


def _mixed(precision="fp64"):
    """Orders 1..12, square and ragged grids, both boundary types, different
    step counts (so the set of running instances shrinks during the run)."""
    base = [
        (11, 1, (20, 20), (X, X)),
        (12, 3, (33, 29), (P, X)),
        (13, 5, (47, 47), (X, X)),
        (14, 9, (24, 24), (P, P)),
        (15, 7, (70, 38), (X, P)),
        (16, 12, (31, 31), (X, X)),
        (17, 2, (65, 66), (X, X)),
    ]
    out = []
    for seed, N, n, bc in base:
        pr = wl.random_medium(seed, N, n[0], t_final=0.25, precision=precision)
        out.append(dataclasses.replace(pr, n=n, bc=bc, name=f"{pr.name}_{n[0]}x{n[1]}"))
    return out


def _single(prob, variant, width, monkeypatch):
    monkeypatch.setenv("STARMAP_CHUNK_WIDTH", str(width))
    s = pa.Solver.from_problem(prob)
    s.set_variant(variant)
    s.run()
    return s.moments()


def _identical(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_batch_equals_single_runs_and_oracle(monkeypatch):
    probs = _mixed()
    solvers = [pa.Solver.from_problem(p) for p in probs]
    steps = [s.nsteps for s in solvers]
    assert len(set(steps)) > 3
    b = pa.Batch(solvers)
    print("batch", [p.name for p in probs], steps, flush=True)
    rec = b.run(use_graph=True)
    assert b.variant() == (0, 8)
    # one launch per sweep and order group, for as long as the group's longest run
    groups = b.groups()
    assert [g["N"] for g in groups] == sorted({p.N for p in probs})
    assert sum(g["count"] for g in groups) == len(probs)
    assert all((g["variant"], g["width"]) == (0, 8) for g in groups)
    assert rec["launches"] == sum(2 * max(n for s, n in zip(solvers, steps) if s.N == g["N"]) + 1 for g in groups)
    assert rec["updates"] == sum(s.nmom * p.n[0] * p.n[1] * n for s, p, n in zip(solvers, probs, steps))
    for s in solvers:
        assert s.time()[2] == s.nsteps
    got = [s.moments() for s in solvers]
    for p, g in zip(probs, got):
        print("single", p.name, flush=True)
        assert _identical(g, _single(p, 0, 8, monkeypatch)), p.name
        o = run_oracle(p, fused=False)
        assert_parity(g, o.u, 1e-12, p.name)
    b.close()


def test_batch_eager_graph_and_rerun_agree():
    probs = _mixed()
    solvers = [pa.Solver.from_problem(p) for p in probs]
    b = pa.Batch(solvers)
    b.run(use_graph=False)
    eager = [s.moments() for s in solvers]
    b.reset()
    assert all(s.time()[2] == 0 for s in solvers)
    b.run(use_graph=True)
    g1 = [s.moments() for s in solvers]
    b.reset()
    b.run(use_graph=True)  # the captured graph is relaunched
    g2 = [s.moments() for s in solvers]
    for e, x, y in zip(eager, g1, g2):
        assert _identical(e, x) and _identical(x, y)
    # a finished batch has nothing left to run
    rec = b.run()
    assert rec["launches"] == 0 and rec["updates"] == 0
    b.close()


@pytest.mark.parametrize("variant,width", [(1, 4), (3, 6), (5, 4), (6, 6), (13, 4)])
def test_batch_tile_variants(variant, width, monkeypatch):
    probs = _mixed()
    solvers = [pa.Solver.from_problem(p) for p in probs]
    b = pa.Batch(solvers)
    b.set_variant(variant, width)
    b.run()
    for p, s in zip(probs[:4], solvers[:4]):
        assert _identical(s.moments(), _single(p, variant, width, monkeypatch)), (p.name, variant, width)
    b.close()


def test_batch_fp32_and_autotune(monkeypatch):
    probs = _mixed("fp32")
    solvers = [pa.Solver.from_problem(p) for p in probs]
    b = pa.Batch(solvers)
    b.autotune(2)
    for g in b.groups():
        assert 0 <= g["variant"] < pa.variant_count() and g["width"] in (4, 6, 8), g
    b.run()
    for i, (p, s) in enumerate(zip(probs, solvers)):
        v, w = b.tile_of(i)
        g = s.moments()
        assert _identical(g, _single(p, v, w, monkeypatch)), (p.name, v, w)
        assert_parity(g, run_oracle(p).u, 1e-5, p.name)
    b.close()


def test_batch_groups_with_their_own_tiles(monkeypatch):
    """Groups of one batch on different tiles: every instance still equals its
    single run on its group's tile, and the run is one graph relaunched."""
    probs = _mixed()
    solvers = [pa.Solver.from_problem(p) for p in probs]
    b = pa.Batch(solvers)
    b.set_variant(0, 8)
    b.run()
    b.reset()
    # a different tile per group (orders 1, 2, 3, 5, 7, 9, 12)
    choice = [(1, 4), (3, 6), (5, 4), (6, 6), (13, 4), (0, 4), (0, 6)]
    for gi, g in enumerate(b.groups()):
        b.set_group_variant(gi, *choice[gi % len(choice)])
    tiles = {g["N"]: (g["variant"], g["width"]) for g in b.groups()}
    assert len(set(tiles.values())) == len(tiles)
    b.run(use_graph=True)
    first = [s.moments() for s in solvers]
    b.reset()
    b.run(use_graph=True)
    for p, s, f in zip(probs, solvers, first):
        assert _identical(s.moments(), f), p.name
        assert _identical(f, _single(p, *tiles[p.N], monkeypatch)), (p.name, tiles[p.N])
    b.close()


def test_merged_launches_equal_chains_and_single_runs(monkeypatch):
    """Merged launches (one launch per sweep over every group, one variant,
    each group its own m-range width) give the same bits as the per-group
    chains and as the single runs; graph and eager, and a relaunched graph."""
    probs = _mixed()
    solvers = [pa.Solver.from_problem(p) for p in probs]
    b = pa.Batch(solvers)
    widths = [4, 6, 8]
    for gi, g in enumerate(b.groups()):
        b.set_group_variant(gi, 11, widths[gi % 3])
    tiles = {g["N"]: (g["variant"], g["width"]) for g in b.groups()}
    b.run()
    chains = [s.moments() for s in solvers]
    b.set_merged(True)
    assert b.merged()
    launches = []
    for use_graph in (True, True, False):
        b.reset()
        rec = b.run(use_graph=use_graph)
        launches.append(rec["launches"])
        for p, s, c in zip(probs, solvers, chains):
            assert _identical(s.moments(), c), (p.name, use_graph)
    # one launch per sweep in total, for as long as the longest instance runs
    assert launches[0] == 2 * max(s.nsteps for s in solvers) + 1
    for p, c in zip(probs, chains):
        assert _identical(c, _single(p, *tiles[p.N], monkeypatch)), p.name
    # a group on another variant turns merging off; merging needs one variant
    b.set_group_variant(0, 0, 8)
    assert not b.merged()
    with pytest.raises(pa.StarmapError):
        b.set_merged(True)
    b.close()


def test_batch_autotune_choice_is_consistent():
    """After the autotuner, merged launches imply one variant for all groups,
    and the run equals the oracle."""
    probs = _mixed("fp32")
    solvers = [pa.Solver.from_problem(p) for p in probs]
    b = pa.Batch(solvers)
    b.autotune(1)
    groups = b.groups()
    if b.merged():
        assert len({g["variant"] for g in groups}) == 1
    b.run()
    for p, s in zip(probs[:3], solvers[:3]):
        assert_parity(s.moments(), run_oracle(p).u, 1e-5, p.name)
    b.close()


def test_batch_rejects_bad_input():
    a = pa.Solver.from_problem(_mixed()[0])
    c = pa.Solver.from_problem(_mixed("fp32")[1])
    with pytest.raises(pa.StarmapError):
        pa.Batch([a, c])  # mixed storage
    with pytest.raises(pa.StarmapError):
        pa.Batch([a, a])
    with pytest.raises(pa.StarmapError):
        pa.Batch([])
    b = pa.Batch([a])
    with pytest.raises(pa.StarmapError):
        b.set_variant(0, 5)
    with pytest.raises(pa.StarmapError):
        b.set_variant(17, 8)
    with pytest.raises(pa.StarmapError):
        b.set_group_variant(1, 0, 8)  # one group only
    b.close()


def test_c4_full_batch_sampled_instances(monkeypatch):
    """The 256-instance FP32 batch at full size, in the launch configuration
    the benchmark times: sampled instances equal their single runs bit for
    bit, the smallest one matches the oracle, and all stay finite."""
    probs = wl.batch(256, "fp32")
    solvers = [pa.Solver.from_problem(p) for p in probs]
    b = pa.Batch(solvers)
    rec = b.run(use_graph=True)
    print("c4", rec, flush=True)
    steps = [s.nsteps for s in solvers]
    sizes = [p.n[0] for p in probs]
    pick = sorted({int(np.argmin(steps)), int(np.argmax(steps)), int(np.argmax([p.N for p in probs]))})
    for i in pick:
        assert _identical(solvers[i].moments(), _single(probs[i], 0, 8, monkeypatch)), probs[i].name
    i = int(np.argmin(sizes))
    assert_parity(solvers[i].moments(), run_oracle(probs[i]).u, 1e-5, probs[i].name)
    for s in solvers:
        d = s.diagnostics()
        assert d["nonfinite"] == 0 and d["maxabs"] > 0
    b.close()


def test_batch_of_filtered_and_anisotropic_instances(monkeypatch):
    """FP_N damping and anisotropic scattering live in per-order decay planes;
    a batch of such instances (mixed with plain ones) equals the single runs
    bitwise and the oracle."""
    probs = _mixed()[:5]
    probs[0] = dataclasses.replace(probs[0], filter_damping=wl.filter_damping(probs[0].N, 6.0, power=2))
    probs[2] = dataclasses.replace(probs[2], filter_damping=wl.filter_damping(probs[2].N, 3.0))
    probs[3] = dataclasses.replace(probs[3], sigma_sl=lambda l, t, x, y: 0.7 ** l + 0 * x)
    solvers = [pa.Solver.from_problem(p) for p in probs]
    b = pa.Batch(solvers)
    b.set_variant(6, 6)
    b.run()
    for p, s in zip(probs, solvers):
        assert _identical(s.moments(), _single(p, 6, 6, monkeypatch)), p.name
        assert_parity(s.moments(), run_oracle(p).u, 1e-12, p.name)
    b.close()
