"""Pins of the oracle's moment matrices, grid classes and time-step rule
against what the paper prints and what the mathematics fixes."""
import math
import os

import numpy as np
import pytest

from oracle import pn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "p3_real_matrices.txt")


def _load_p3_golden():
    M = {"Mx": np.zeros((10, 10)), "My": np.zeros((10, 10))}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, r, c, sign, p, q = line.split()
            M[name][int(r), int(c)] = (1.0 if sign == "+" else -1.0) * math.sqrt(int(p) / int(q)) / 2.0
    return M["Mx"], M["My"]


def test_p3_matrices_match_printed_entries():
    """Every entry (zeros included) of the printed P_3 M_x and M_y (Sect. 3)."""
    gx, gy = _load_p3_golden()
    Mx, My = pn.real_matrices(3)
    assert Mx.shape == (10, 10)
    np.testing.assert_allclose(Mx, gx, rtol=0, atol=1e-15)
    np.testing.assert_allclose(My, gy, rtol=0, atol=1e-15)


def test_moment_order_p3():
    assert pn.moments(3) == [("R", 0, 0), ("R", 1, 1), ("I", 1, 1), ("R", 2, 2), ("I", 2, 2),
                             ("R", 2, 0), ("R", 3, 3), ("I", 3, 3), ("R", 3, 1), ("I", 3, 1)]


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 9, 15, 39])
def test_transformation_unitary_and_matrices_real_symmetric(N):
    S = pn.transformation(N)
    np.testing.assert_allclose(S @ S.conj().T, np.eye(S.shape[0]), atol=1e-15)
    Mx, My = pn.real_matrices(N)
    assert Mx.shape == ((N + 1) * (N + 2) // 2,) * 2
    np.testing.assert_allclose(Mx, Mx.T, atol=1e-15)  # symmetric (eq. real_valued_pn_equations)
    np.testing.assert_allclose(My, My.T, atol=1e-15)
    # at most four nonzeros per row of each matrix (Sect. 5.5)
    assert np.max(np.count_nonzero(Mx, axis=1)) <= 4
    assert np.max(np.count_nonzero(My, axis=1)) <= 4


@pytest.mark.parametrize("N", [3, 7, 13])
def test_lemma2_coupling_pattern(N):
    """M_x couples R<->R and I<->I, M_y couples R<->I, and only orders l +- 1,
    m +- 1 (Lemma 2)."""
    Mx, My = pn.real_matrices(N)
    mom = pn.moments(N)
    for i, (ki, li, mi) in enumerate(mom):
        for j, (kj, lj, mj) in enumerate(mom):
            if Mx[i, j] != 0:
                assert ki == kj and abs(li - lj) == 1 and abs(mi - mj) == 1
            if My[i, j] != 0:
                assert ki != kj and abs(li - lj) == 1 and abs(mi - mj) == 1


@pytest.mark.parametrize("N", list(range(1, 40)))
def test_spectral_radius_is_largest_legendre_root(N):
    """rho(M_x) equals the largest root of P_{N+1}; the spectrum lies in (-1, 1)."""
    Mx, _ = pn.real_matrices(N)
    nodes, _ = np.polynomial.legendre.leggauss(N + 1)
    ev = np.linalg.eigvalsh(Mx)
    assert np.all(np.abs(ev) < 1.0)
    assert abs(pn.spectral_radius(Mx) - np.max(nodes)) < 1e-12


@pytest.mark.parametrize("N", [3, 6, 11])
def test_rotational_invariance_of_spectrum(N):
    """eig(cos t M_x + sin t M_y) = eig(M_x) (Sect. 5.3 assumption)."""
    Mx, My = pn.real_matrices(N)
    ref = np.sort(np.linalg.eigvalsh(Mx))
    for th in (0.3, 1.1, 2.5):
        ev = np.sort(np.linalg.eigvalsh(math.cos(th) * Mx + math.sin(th) * My))
        np.testing.assert_allclose(ev, ref, atol=1e-13)


@pytest.mark.parametrize("N", [1, 4, 9, 39])
def test_slab_eigenvalues_are_gauss_legendre_nodes(N):
    M = pn.slab_matrix(N)
    nodes, _ = np.polynomial.legendre.leggauss(N + 1)
    ev = np.sort(np.linalg.eigvals(M).real)
    np.testing.assert_allclose(ev, np.sort(nodes), atol=1e-12)


COUNTS = {  # N: (N_mom, G11, G22, G21, G12)
    1: (3, 1, 0, 1, 1), 3: (10, 3, 1, 3, 3), 5: (21, 6, 3, 6, 6), 7: (36, 10, 6, 10, 10),
    9: (55, 15, 10, 15, 15), 31: (528, 136, 120, 136, 136), 39: (820, 210, 190, 210, 210)}


@pytest.mark.parametrize("N", sorted(COUNTS))
def test_grid_classes(N):
    """Greedy assignment (Sect. 5.3) = R/I and parity rule; conditions of
    eq. (matrix_conditions) hold; class sizes."""
    Mx, My = pn.real_matrices(N)
    gx, gy = pn.grid_classes(Mx, My)
    for k, (kind, l, m) in enumerate(pn.moments(N)):
        if kind == "R":
            want = (1, 1) if l % 2 == 0 else (2, 1)
        else:
            want = (2, 2) if l % 2 == 0 else (1, 2)
        assert (gx[k], gy[k]) == want
        # even components (I11 u I22) are exactly the even orders
        assert pn.is_even_component(gx[k], gy[k]) == (l % 2 == 0)
    nmom, c11, c22, c21, c12 = COUNTS[N]
    g = list(zip(gx, gy))
    assert len(g) == nmom
    assert (g.count((1, 1)), g.count((2, 2)), g.count((2, 1)), g.count((1, 2))) == (c11, c22, c21, c12)
    n = len(g)
    for i in range(n):
        for j in range(n):
            if Mx[i, j] != 0:
                assert (g[i], g[j]) in {((1, 1), (2, 1)), ((2, 1), (1, 1)), ((1, 2), (2, 2)), ((2, 2), (1, 2))}
            if My[i, j] != 0:
                assert (g[i], g[j]) in {((1, 1), (1, 2)), ((1, 2), (1, 1)), ((2, 1), (2, 2)), ((2, 2), (2, 1))}


def _swap_permutation(N):
    """Signed permutation for the x<->y reflection of the angular variable."""
    mom = pn.moments(N)
    idx = {t: i for i, t in enumerate(mom)}
    P = np.zeros((len(mom), len(mom)))
    for i, (kind, l, m) in enumerate(mom):
        if m % 2 == 0:
            s = (-1.0) ** (m // 2)
            P[i, i] = s if kind == "R" else -s
        else:
            s = (-1.0) ** ((m - 1) // 2)
            P[i, idx[("I" if kind == "R" else "R", l, m)]] = s
    return P


@pytest.mark.parametrize("N", [3, 7, 39])
def test_reflection_symmetries_of_matrices(N):
    """x<->y swap P: P M_x P^T = M_y; x-mirror Q: Q M_x Q^T = -M_x, Q M_y Q^T = M_y."""
    Mx, My = pn.real_matrices(N)
    P = _swap_permutation(N)
    np.testing.assert_allclose(P @ Mx @ P.T, My, atol=1e-14)
    np.testing.assert_allclose(P @ My @ P.T, Mx, atol=1e-14)
    q = np.array([((-1.0) ** m if kind == "R" else -((-1.0) ** m)) for kind, l, m in pn.moments(N)])
    Q = np.diag(q)
    np.testing.assert_allclose(Q @ Mx @ Q.T, -Mx, atol=1e-14)
    np.testing.assert_allclose(Q @ My @ Q.T, My, atol=1e-14)


def test_time_step_rule():
    rho = 0.8611363115940526
    dt, n = pn.time_step(0.5, 0.03, 0.03, rho, 1.0)
    assert n == 58 and abs(dt - 1.0 / 58) < 1e-16
    # lands exactly on t_final; dt never exceeds the CFL bound
    for h in (0.003, 0.025, 0.01):
        dt, n = pn.time_step(0.5, h, h, rho, 1.7)
        assert dt <= 0.5 * h / rho * (1 + 1e-12) and abs(n * dt - 1.7) < 1e-12
