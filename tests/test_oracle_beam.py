"""Beam problem (a source q(x) delta(Omega - Omega_0)): pins of the oracle's
direction moments, the library's own values against them, and the oracle's
exact mass growth."""
import math

import numpy as np
import pytest

import paper_1211_2205_amd as pa
import workloads as wl
from oracle import pn
from oracle.scheme import OracleSolver

DIRS = [(math.cos(math.pi / 6), math.sin(math.pi / 6), 0.0), (0.0, 1.0, 0.0), (-1.0, 0.0, 0.0),
        (0.48, -0.6, 0.64), (0.0, 0.0, 1.0), (0.1, 0.2, -math.sqrt(0.95))]


def test_low_order_values_are_the_printed_moments():
    # R_0^0 = (4 pi)^(-1/2) int psi, R_1^1 = sqrt(3/(4 pi)) int Omega_x psi,
    # I_1^1 = sqrt(3/(4 pi)) int Omega_y psi (Sect. 3)
    for om in DIRS:
        phi = pn.direction_moments(3, om)
        assert abs(phi[0] - 1 / math.sqrt(4 * math.pi)) < 1e-15
        assert abs(phi[1] - math.sqrt(3 / (4 * math.pi)) * om[0]) < 1e-15
        assert abs(phi[2] - math.sqrt(3 / (4 * math.pi)) * om[1]) < 1e-15


@pytest.mark.parametrize("N", list(range(1, 13)) + [39])
def test_recursion_of_the_basis(N):
    """Omega phi_k = sum_j M(k, j) phi_j for every row below the top order:
    the real moment matrices are the recursion of the basis they act on."""
    Mx, My = pn.real_matrices(N)
    low = [k for k, (_, l, _) in enumerate(pn.moments(N)) if l < N]
    for om in DIRS:
        phi = pn.direction_moments(N, om)
        np.testing.assert_allclose((Mx @ phi)[low], om[0] * phi[low], rtol=0, atol=2e-13)
        np.testing.assert_allclose((My @ phi)[low], om[1] * phi[low], rtol=0, atol=2e-13)


@pytest.mark.parametrize("N", [4, 9])
def test_basis_is_orthonormal_on_the_sphere(N):
    # Gauss-Legendre in mu (exact for the polynomial part), uniform in azimuth
    mus, wmu = np.polynomial.legendre.leggauss(N + 2)
    nphi = 2 * N + 3
    G = np.zeros((pn.moments(N).__len__(),) * 2)
    for mu, w in zip(mus, wmu):
        s = math.sqrt(1 - mu * mu)
        for j in range(nphi):
            ph = 2 * math.pi * j / nphi
            v = pn.direction_moments(N, (s * math.cos(ph), s * math.sin(ph), mu))
            G += w * (2 * math.pi / nphi) * np.outer(v, v)
    np.testing.assert_allclose(G, np.eye(len(G)), rtol=0, atol=1e-12)


@pytest.mark.parametrize("N", [1, 3, 9, 39, 60])
def test_library_direction_moments_match_oracle(N):
    for om in DIRS:
        np.testing.assert_allclose(pa.direction_moments(N, om), pn.direction_moments(N, om), rtol=0, atol=1e-13)
    with pytest.raises(pa.StarmapError):
        pa.direction_moments(N, (1.0, 1.0, 0.0))


def test_oracle_beam_mass_grows_linearly():
    """No absorption anywhere: the zeroth moment gains dt * sum(q_0) per step
    exactly while no radiation reaches the boundary."""
    prob = wl.beam(N=3, n=40, t_final=0.2)
    o = OracleSolver(prob)
    o.evaluate_materials(0.0)
    q0 = o.grid.dx * o.grid.dy * float(np.sum(o._q[0]))
    assert abs(q0 - 1 / math.sqrt(4 * math.pi)) < 1e-3  # unit-mass Gaussian times phi_0
    o.run(fused=True)
    assert abs(o.mass() - o.t * q0) < 1e-12 * o.t * q0
