"""Pins of the closure oracle (network, features, targets, closure solver)
against what mathematics and independent routines fix."""
import math

import numpy as np
import pytest
import torch
from scipy.stats import norm

import workloads as wl
from oracle import closure as oc
from oracle import mlp, pn
from oracle.scheme import OracleSolver


def _toy(seed=0, n_in=6, n_hidden=5, n_out=3, batch=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = mlp.init(n_in, n_hidden, n_out, seed)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(size=p[k].shape) * 0.3
    X = rng.normal(size=(batch, n_in))
    T = rng.normal(size=(batch, n_out))
    return p, X, T


def test_gelu_is_x_times_normal_cdf():
    z = np.linspace(-8, 8, 401)
    np.testing.assert_allclose(mlp.gelu(z), z * norm.cdf(z), rtol=0, atol=1e-15)
    # gelu(-z) = gelu(z) - z because Phi(-z) = 1 - Phi(z)
    np.testing.assert_allclose(mlp.gelu(-z), mlp.gelu(z) - z, rtol=0, atol=1e-14)


def test_gelu_grad_matches_central_differences():
    z = np.linspace(-6, 6, 121)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, rtol=0, atol=1e-9)


def test_backward_matches_central_differences():
    p, X, T = _toy()
    Y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, Y, T)
    h = 1e-6
    for name in mlp.NAMES:
        fd = np.zeros_like(p[name])
        for idx in np.ndindex(p[name].shape):
            keep = p[name][idx]
            p[name][idx] = keep + h
            lp = mlp.loss(mlp.forward(p, X)[0], T)
            p[name][idx] = keep - h
            lm = mlp.loss(mlp.forward(p, X)[0], T)
            p[name][idx] = keep
            fd[idx] = (lp - lm) / (2 * h)
        err = np.max(np.abs(g[name] - fd)) / max(np.max(np.abs(fd)), 1e-30)
        assert err < 1e-7, (name, err)


def test_bf16_rounding_matches_torch():
    rng = np.random.Generator(np.random.PCG64(3))
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-20, 20, size=4000),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20]])
    x32 = x.astype(np.float32)  # exactly representable inputs for torch
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x32.astype(np.float64)), ref)
    # ties go to even; above the tie rounds up
    assert mlp.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0
    assert mlp.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    assert mlp.bf16_round(np.array([1 + 2 ** -8 + 2 ** -20]))[0] == 1 + 2 ** -7


def test_bf16_backward_reduces_to_fp64_on_representable_values():
    # when every operand is already a bfloat16 value the rounding is the identity
    p, X, T = _toy(seed=5)
    for k in ("W1", "W2", "W3"):
        p[k] = mlp.bf16_round(p[k])
    X = mlp.bf16_round(X)
    Y, c = mlp.forward(p, X, bf16=False)
    Yb, cb = mlp.forward(p, X, bf16=True)
    # a1, a2 are rounded in the bf16 network only, so compare to a looser bound
    assert np.max(np.abs(Y - Yb)) < 1e-2 * np.max(np.abs(Y))
    g = mlp.backward(p, c, Y, T)
    gb = mlp.backward(p, cb, Yb, T, bf16=True)
    for k in mlp.NAMES:
        assert np.max(np.abs(g[k] - gb[k])) <= 3e-2 * np.max(np.abs(g[k])) + 1e-12, k


def test_adam_first_step_and_convergence():
    rng = np.random.Generator(np.random.PCG64(9))
    target = {"w": rng.normal(size=5)}
    p = {"w": np.zeros(5)}
    opt = mlp.Adam(p, lr=0.01)
    g = {"w": p["w"] - target["w"]}
    p1 = opt.step({"w": p["w"].copy()}, g)
    # first step: mhat = g, vhat = g^2, so the step is lr * g / (|g| + eps)
    np.testing.assert_allclose(p1["w"], -0.01 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=1e-12, atol=0)
    p = p1
    for _ in range(5000):
        p = opt.step(p, {"w": p["w"] - target["w"]})
    np.testing.assert_allclose(p["w"], target["w"], atol=1e-6)


def test_flatten_roundtrip_and_blob_size():
    p = mlp.init(oc.N_IN, oc.N_HIDDEN, oc.N_OUT, 1, fan_in=oc.N_FEATURES)
    f = mlp.flatten(p)
    assert f.size == 128 * 128 + 128 + 128 * 128 + 128 + 6 * 128 + 6 == 33798
    q = mlp.unflatten(f, oc.N_IN, oc.N_HIDDEN, oc.N_OUT)
    for k in mlp.NAMES:
        np.testing.assert_array_equal(p[k], q[k])
    assert np.all(p["W1"][:, oc.N_FEATURES:] == 0)


def test_closure_moments_are_orders_4_and_5():
    inputs, outputs = oc.closure_moments()
    assert [(k, l, m) for k, l, m in inputs] == [
        ("R", 4, 4), ("I", 4, 4), ("R", 4, 2), ("I", 4, 2), ("R", 4, 0),
        ("R", 5, 5), ("I", 5, 5), ("R", 5, 3), ("I", 5, 3), ("R", 5, 1), ("I", 5, 1)]
    assert outputs == inputs[5:]


def _small(N, n=(9, 7), seed=3):
    prob = wl.random_medium(seed, N, n[0], precision="fp64")
    prob.n = n
    return prob


def test_features_gather_clamped_stencils_brute_force():
    s = OracleSolver(_small(7))
    inputs, _ = oc.closure_moments()
    idx = [s.moms.index(km) for km in inputs]
    for p, k in enumerate(idx):
        ny, nx = s.u[k].shape
        J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        s.u[k][:] = 1000.0 * (p + 1) + 10.0 * J + I
    pts = [(0, 0), (4, 3), (9, 7), (9, 0), (0, 7), (8, 6)]
    X, nu = oc.features(s, pts)
    for r, (i, j) in enumerate(pts):
        vals = []
        for p, k in enumerate(idx):
            ny, nx = s.u[k].shape
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    jj = j + b
                    ii = i + a
                    jj = 0 if jj < 0 else (ny - 1 if jj > ny - 1 else jj)
                    ii = 0 if ii < 0 else (nx - 1 if ii > nx - 1 else ii)
                    vals.append(1000.0 * (p + 1) + 10.0 * jj + ii)
        vals = np.array(vals)
        assert abs(nu[r] - math.sqrt(np.sum(vals ** 2))) < 1e-9 * nu[r]
        np.testing.assert_allclose(X[r, :99] * nu[r], vals, rtol=1e-14)
        assert np.all(X[r, 101:] == 0)
        # sigma of the G11 cell (clamped)
        ci, cj = min(i, 8), min(j, 6)
        Xc, Yc = s.grid.coords(1, 1)
        sa = s.prob.sigma_a(0, Xc[cj, ci], Yc[cj, ci])
        assert abs(X[r, 99] - math.log10(sa + 0.01)) < 1e-14


def test_order6_flux_of_linear_fields_is_exact_in_the_interior():
    # u_j = a_j x + b_j y on the order-6 moments: every difference is exact
    # away from the boundary, so F_k = -sum_j (Mx(k,j) a_j + My(k,j) b_j)
    s = OracleSolver(_small(7, n=(12, 10)))
    rng = np.random.Generator(np.random.PCG64(4))
    coef = {}
    for k, (kind, l, m) in enumerate(s.moms):
        if l == 6:
            a, b = rng.normal(size=2)
            coef[k] = (a, b)
            X, Y = s.grid.coords(s.gx[k], s.gy[k])
            s.u[k][:] = a * X + b * Y
        else:
            s.u[k][:] = rng.normal(size=s.u[k].shape)  # must not enter F
    W = oc.order6_flux(s)
    for k, (kind, l, m) in enumerate(s.moms):
        if l != 5:
            continue
        exp = -sum(s.Mx[k, j] * ab[0] + s.My[k, j] * ab[1] for j, ab in coef.items())
        np.testing.assert_allclose(W[k][2:-2, 2:-2], exp, rtol=0, atol=1e-12)


def test_order6_flux_is_the_truncation_gap():
    # W of the full P_7 odd residual minus that of the state without order 6
    s = OracleSolver(_small(7))
    rng = np.random.Generator(np.random.PCG64(6))
    for a in s.u:
        a[:] = rng.normal(size=a.shape)
    full = s.flux(1)
    keep = [a.copy() for a in s.u]
    for k, (kind, l, m) in enumerate(s.moms):
        if l == 6:
            s.u[k][:] = 0
    cut = s.flux(1)
    s.u = keep
    F = oc.order6_flux(s)
    for k, (kind, l, m) in enumerate(s.moms):
        if l == 5:
            np.testing.assert_allclose(F[k], full[k] - cut[k], rtol=0, atol=1e-12)


def test_zero_output_layer_gives_plain_p5():
    prob = _small(5, n=(11, 11))
    p = mlp.init(oc.N_IN, oc.N_HIDDEN, oc.N_OUT, 2, fan_in=oc.N_FEATURES)
    p["W3"][:] = 0
    p["b3"][:] = 0
    c = oc.ClosureSolver(prob, p)
    c.advance(4)
    o = OracleSolver(prob)
    o.advance(4, fused=True)
    for a, b in zip(c.u, o.u):
        np.testing.assert_array_equal(a, b)


def test_closure_terms_are_scale_equivariant():
    prob = _small(5, n=(8, 8))
    p = mlp.init(oc.N_IN, oc.N_HIDDEN, oc.N_OUT, 4, fan_in=oc.N_FEATURES)
    s = OracleSolver(prob)
    rng = np.random.Generator(np.random.PCG64(1))
    for a in s.u:
        a[:] = rng.normal(size=a.shape)
    G1 = oc.closure_terms(s, p)
    for a in s.u:
        a *= 8.0
    G8 = oc.closure_terms(s, p)
    for k in G1:
        np.testing.assert_allclose(G8[k], 8.0 * G1[k], rtol=1e-13, atol=0)
