"""Seeded synthetic problem descriptions for the staggered-grid P_N solver.

This module only describes *inputs*: domain, grid size, moment order, boundary
type, CFL number, final time, and the material / source / initial-condition
fields as vectorised functions f(t, x, y) of physical coordinates.  It holds
none of the scheme's arithmetic (no moment matrices, no staggered grids, no
time step rule); the oracle and the GPU library each sample these functions on
their own grids.

The problems follow the paper's workloads (Sect. 6):
  * line source   (Sect. 6.4): isotropic Gaussian of the zeroth moment in a
    purely scattering medium, sigma_s0 = 1;
  * checkerboard  (Sect. 6.3): [0,7]^2 lattice with unit absorbing blocks,
    isotropic unit source in [3,4]^2, scattering elsewhere;
  * heterogeneous batch / closure instances: random 8x8 piecewise-constant
    materials with a Gaussian source (no counterpart in the paper; the recipe
    is stated in the design notes).
Moment index 0 is the zeroth moment R_0^0 (the paper's first component).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, Optional, Sequence

import numpy as np

Field = Callable[[float, np.ndarray, np.ndarray], np.ndarray]

BC_PERIODIC = "periodic"
BC_EXTRAPOLATION = "extrapolation"


@dataclasses.dataclass
class Problem:
    """Problem statement (the paper's ``par`` struct, Sect. 5.1)."""

    name: str
    N: int                       # moment order
    n: tuple                     # (nx, ny) cells
    ax: tuple                    # (x0, x1, y0, y1)
    bc: tuple                    # per axis: BC_PERIODIC or BC_EXTRAPOLATION
    cfl: float
    t_final: float
    sigma_a: Field
    sigma_s0: Field
    # anisotropic part: sigma_sl(l, t, x, y) for l >= 1, or None (isotropic)
    sigma_sl: Optional[Callable[[int, float, np.ndarray, np.ndarray], np.ndarray]] = None
    source: Dict[int, Field] = dataclasses.field(default_factory=dict)
    initial: Dict[int, Field] = dataclasses.field(default_factory=dict)
    time_dependent: bool = False  # materials / sources depend on t
    precision: str = "fp64"
    seed: Optional[int] = None
    # beam source q(x) delta(Omega - Omega_0): unit direction Omega_0 and q(x);
    # each solver turns it into moment sources with its own basis values
    beam_direction: Optional[tuple] = None
    beam_profile: Optional[Field] = None
    # time-separable form of some fields: {"absorption": [(a, g), ...],
    # "scattering": [...], "scattering_order": {l: [...]}, "source": {k: [...]}}
    # with a(t) a float and g(x, y) an array; the listed fields equal
    # sum a(t) g(x, y) (the callables above give the same values)
    separable: Optional[dict] = None
    # filtered P_N: damping d_l (l = 0..N) added to the decay of every order-l moment
    filter_damping: Optional[Sequence[float]] = None
    # diffusion-corrected P_N: coefficient kappa(x, y) of the diffusion step on
    # the order-N moments (time-independent; called with t = 0)
    diffusion: Optional[Field] = None

    @property
    def nmom(self) -> int:
        return (self.N + 1) * (self.N + 2) // 2


def _const(v: float) -> Field:
    def f(t, x, y):
        return np.full(np.broadcast(x, y).shape, float(v))
    return f


def _zero(t, x, y):
    return np.zeros(np.broadcast(x, y).shape)


def gaussian_std(s: float, xc: float = 0.0, yc: float = 0.0) -> Field:
    """Unit-mass isotropic Gaussian of standard deviation s."""
    def f(t, x, y):
        r2 = (np.asarray(x) - xc) ** 2 + (np.asarray(y) - yc) ** 2
        return np.exp(-r2 / (2.0 * s * s)) / (2.0 * math.pi * s * s)
    return f


def gaussian_pseudo_time(sigma: float) -> Field:
    """The paper's Gaussian written with a pseudo-time sigma (Sect. 6.4):
    1/(4 pi sigma) exp(-r^2 / (4 sigma))."""
    def f(t, x, y):
        r2 = np.asarray(x) ** 2 + np.asarray(y) ** 2
        return np.exp(-r2 / (4.0 * sigma)) / (4.0 * math.pi * sigma)
    return f


# --------------------------------------------------------------------------
# Line source (Sect. 6.4), synthetic sizes of the benchmark configurations.
# --------------------------------------------------------------------------
def line_source(N: int = 3, n: int = 100, s: float = 0.03, half_width: float = 1.5,
                t_final: float = 1.0, cfl: float = 0.5, precision: str = "fp64",
                bc: str = BC_EXTRAPOLATION) -> Problem:
    return Problem(
        name=f"line_source_P{N}_{n}",
        N=N, n=(n, n), ax=(-half_width, half_width, -half_width, half_width),
        bc=(bc, bc), cfl=cfl, t_final=t_final,
        sigma_a=_zero, sigma_s0=_const(1.0),
        initial={0: gaussian_std(s)}, precision=precision)


# --------------------------------------------------------------------------
# Checkerboard lattice (Sect. 6.3).  Unit block (i, j) covers [i, i+1) x [j, j+1).
# Absorbers: i, j in 1..5 with i + j even, except the source block (3, 3) and
# the open block (3, 5) above it: eleven absorbing unit squares.
# --------------------------------------------------------------------------
CHECKER_ABSORBERS = tuple(
    (i, j) for i in range(1, 6) for j in range(1, 6)
    if (i + j) % 2 == 0 and (i, j) not in ((3, 3), (3, 5)))


def _block_index(v: np.ndarray) -> np.ndarray:
    # points that lie on a block edge belong to the block above (half-open
    # blocks); the small offset absorbs round-off in the sampled coordinate
    return np.floor(np.asarray(v, dtype=np.float64) + 1e-9).astype(np.int64)


def _checker_absorber_mask(x, y):
    bi, bj = _block_index(x), _block_index(y)
    m = np.zeros(np.broadcast(bi, bj).shape, dtype=bool)
    for (i, j) in CHECKER_ABSORBERS:
        m |= (bi == i) & (bj == j)
    return m


def checkerboard(N: int = 7, n: int = 280, t_final: float = 3.2, cfl: float = 0.5,
                 precision: str = "fp64") -> Problem:
    def sig_a(t, x, y):
        return np.where(_checker_absorber_mask(x, y), 10.0, 0.0)

    def sig_s(t, x, y):
        return np.where(_checker_absorber_mask(x, y), 0.0, 1.0)

    def src(t, x, y):
        bi, bj = _block_index(x), _block_index(y)
        return np.where((bi == 3) & (bj == 3), 1.0, 0.0)

    return Problem(
        name=f"checkerboard_P{N}_{n}", N=N, n=(n, n), ax=(0.0, 7.0, 0.0, 7.0),
        bc=(BC_EXTRAPOLATION, BC_EXTRAPOLATION), cfl=cfl, t_final=t_final,
        sigma_a=sig_a, sigma_s0=sig_s, source={0: src}, precision=precision)


# --------------------------------------------------------------------------
# Random heterogeneous instances (batched solves and the learned closure).
# Domain [-1,1]^2, extrapolation; 8x8 blocks of width 0.25 with sigma_a and
# sigma_s log-uniform in [0.1, 10]; isotropic Gaussian source
# exp(-|x - xc|^2 / (2 s^2)), xc ~ U([-0.5,0.5]^2), s ~ U(0.05, 0.2); zero IC.
# --------------------------------------------------------------------------
BATCH_SEED0 = 12112205
CLOSURE_SEED0 = 1_000_000


def _block_field(values: np.ndarray, x0: float, width: float) -> Field:
    nb = values.shape[0]

    def f(t, x, y):
        bi = np.clip(np.floor((np.asarray(x) - x0) / width + 1e-9).astype(np.int64), 0, nb - 1)
        bj = np.clip(np.floor((np.asarray(y) - x0) / width + 1e-9).astype(np.int64), 0, nb - 1)
        return values[bj, bi]
    return f


def random_medium(seed: int, N: int, n: int, t_final: float = 0.5, cfl: float = 0.5,
                  precision: str = "fp32") -> Problem:
    rng = np.random.Generator(np.random.PCG64(seed))
    sa = 10.0 ** rng.uniform(-1.0, 1.0, size=(8, 8))
    ss = 10.0 ** rng.uniform(-1.0, 1.0, size=(8, 8))
    xc, yc = rng.uniform(-0.5, 0.5, size=2)
    s = rng.uniform(0.05, 0.2)

    def src(t, x, y):
        r2 = (np.asarray(x) - xc) ** 2 + (np.asarray(y) - yc) ** 2
        return np.exp(-r2 / (2.0 * s * s))

    return Problem(
        name=f"random_medium_s{seed}_P{N}_{n}", N=N, n=(n, n), ax=(-1.0, 1.0, -1.0, 1.0),
        bc=(BC_EXTRAPOLATION, BC_EXTRAPOLATION), cfl=cfl, t_final=t_final,
        sigma_a=_block_field(sa, -1.0, 0.25), sigma_s0=_block_field(ss, -1.0, 0.25),
        source={0: src}, precision=precision, seed=seed)


def beam(N: int = 9, n: int = 150, t_final: float = 0.6, s: float = 0.03, cfl: float = 0.5,
         precision: str = "fp64") -> Problem:
    """Beam in void and medium (Sect. 6): domain [-0.6, 0.6]^2, extrapolation
    on all sides; void (sigma_t = 0) for x < 0.3; for x >= 0.3 no absorption
    and Henyey-Greenstein scattering sigma_sl = 100 g^l, g = 0.85; a source
    q(x) delta(Omega - Omega_0) with Omega_0 in the plane at angle pi/6 to the
    x-axis and q the Gaussian of the line source (standard deviation s, unit
    mass) at the origin; zero initial state."""
    def medium(x):
        return np.asarray(x) >= 0.3

    def sig_a(t, x, y):
        return np.zeros_like(np.asarray(x, dtype=np.float64))

    def sig_s0(t, x, y):
        return np.where(medium(x), 100.0, 0.0)

    def sig_sl(l, t, x, y):
        return np.where(medium(x), 100.0 * 0.85 ** l, 0.0)

    ang = math.pi / 6.0
    return Problem(
        name=f"beam_P{N}_{n}", N=N, n=(n, n), ax=(-0.6, 0.6, -0.6, 0.6),
        bc=(BC_EXTRAPOLATION, BC_EXTRAPOLATION), cfl=cfl, t_final=t_final,
        sigma_a=sig_a, sigma_s0=sig_s0, sigma_sl=sig_sl, precision=precision,
        beam_direction=(math.cos(ang), math.sin(ang), 0.0), beam_profile=gaussian_std(s))


def _sum_of_terms(terms) -> Field:
    def f(t, x, y):
        out = np.zeros(np.broadcast(x, y).shape)
        for a, g in terms:
            out = out + a(t) * g(x, y)
        return out
    return f


def manufactured(n: int = 32, precision: str = "fp64", t_final: float = 0.5) -> Problem:
    """Manufactured solution of Sect. 6.1 in time-separable form: P_3 on
    [0,1]^2, periodic, sigma_a = t cos(2 pi y), sigma_s0 = 1,
    sigma_sl = 0.9^l, exact R_0^0 = e^-t sin^2(2 pi x), every other moment
    zero; the source is q_0 = R_0^0 (sigma_a - 1) and
    q_1 = c d/dx R_0^0 with c = 1/sqrt(3) the coupling of R_1^1 to R_0^0 in
    M_x of P_3 (the moment with index 1 is R_1^1)."""
    c = math.sqrt(2.0) * math.sqrt(2.0 / 3.0) / 2.0
    two_pi = 2.0 * math.pi
    sep = {
        "absorption": [(lambda t: t, lambda x, y: np.cos(two_pi * y) + 0 * x)],
        "source": {
            0: [(lambda t: t * math.exp(-t), lambda x, y: np.sin(two_pi * x) ** 2 * np.cos(two_pi * y)),
                (lambda t: -math.exp(-t), lambda x, y: np.sin(two_pi * x) ** 2 + 0 * y)],
            1: [(lambda t: math.exp(-t), lambda x, y: c * two_pi * np.sin(2 * two_pi * x) + 0 * y)],
        },
    }
    exact = lambda t, x, y: math.exp(-t) * np.sin(two_pi * x) ** 2 + 0 * y
    return Problem(
        name=f"manufactured_P3_{n}", N=3, n=(n, n), ax=(0.0, 1.0, 0.0, 1.0), bc=(BC_PERIODIC, BC_PERIODIC),
        cfl=0.5, t_final=t_final, sigma_a=_sum_of_terms(sep["absorption"]), sigma_s0=_const(1.0),
        sigma_sl=lambda l, t, x, y: np.full(np.broadcast(x, y).shape, 0.9 ** l),
        source={k: _sum_of_terms(v) for k, v in sep["source"].items()}, initial={0: exact},
        time_dependent=True, precision=precision, separable=sep)


def pulsed_medium(seed: int, N: int, n: int, t_final: float = 0.4, precision: str = "fp64") -> Problem:
    """Heterogeneous time-dependent medium in separable form (no counterpart
    in the paper; a stress case for time-dependent data): on [-1,1]^2 with
    extrapolation boundaries, absorption = 8x8 random blocks in [0,2] plus
    three oscillating terms (1 + sin(w t + p)) times random blocks in [0,1],
    scattering = random blocks in [0,5] times (1 + t/2), anisotropic
    scattering sigma_sl = g^l times the scattering blocks times (1 - t/4)
    with g = 0.6, and a zeroth-moment source of two Gaussian pulses e^-(t-tc)^2/w^2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    blocks = lambda hi: _block_field(rng.uniform(0.0, hi, size=(8, 8)), -1.0, 0.25)
    base = blocks(2.0)
    absorption = [(lambda t: 1.0, lambda x, y, f=base: f(0.0, x, y))]
    for _ in range(3):
        w, p, f = rng.uniform(5.0, 20.0), rng.uniform(0.0, 2 * math.pi), blocks(1.0)
        absorption.append((lambda t, w=w, p=p: 1.0 + math.sin(w * t + p), lambda x, y, f=f: f(0.0, x, y)))
    fs = blocks(5.0)
    scattering = [(lambda t: 1.0 + 0.5 * t, lambda x, y: fs(0.0, x, y))]
    order = {l: [(lambda t: 1.0 - 0.25 * t, lambda x, y, l=l: 0.6 ** l * fs(0.0, x, y))] for l in range(1, N + 1)}
    src = []
    for _ in range(2):
        cx, cy, tc = rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(0.0, t_final)
        g = gaussian_std(0.1, cx, cy)
        src.append((lambda t, tc=tc: math.exp(-((t - tc) / 0.1) ** 2), lambda x, y, g=g: g(0.0, x, y)))
    sep = {"absorption": absorption, "scattering": scattering, "scattering_order": order, "source": {0: src}}
    return Problem(
        name=f"pulsed_medium_s{seed}_P{N}_{n}", N=N, n=(n, n), ax=(-1.0, 1.0, -1.0, 1.0),
        bc=(BC_EXTRAPOLATION, BC_EXTRAPOLATION), cfl=0.5, t_final=t_final,
        sigma_a=_sum_of_terms(absorption), sigma_s0=_sum_of_terms(scattering),
        sigma_sl=lambda l, t, x, y: _sum_of_terms(order[l])(t, x, y), source={0: _sum_of_terms(src)},
        time_dependent=True, precision=precision, seed=seed, separable=sep)


def filter_damping(N: int, strength: float, power: int = 4) -> list:
    """Per-order damping of an exponential-type filter of the given strength:
    d_l = strength (l / (N + 1))^power, l = 0..N."""
    return [strength * (l / (N + 1.0)) ** power for l in range(N + 1)]


def batch_instance(i: int, precision: str = "fp32") -> Problem:
    """Instance i of the 256-instance heterogeneous batch: side n ~ U{64..512},
    N ~ U{3,5,7,9}, drawn from the instance's own seed."""
    seed = BATCH_SEED0 + i
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(64, 513))
    N = int(rng.choice([3, 5, 7, 9]))
    return random_medium(seed + 7_000_000, N, n, precision=precision)


def batch(count: int = 256, precision: str = "fp32") -> Sequence[Problem]:
    return [batch_instance(i, precision) for i in range(count)]


def closure_instance(k: int, N: int, n: int = 256, precision: str = "fp32") -> Problem:
    """Closure training (k < 2000) and held-out evaluation (k >= 2000) instance."""
    return random_medium(CLOSURE_SEED0 + k, N, n, precision=precision)


# --------------------------------------------------------------------------
# The benchmark configurations by name.
# --------------------------------------------------------------------------
def config(name: str, precision: Optional[str] = None) -> Problem:
    if name == "c1":
        return line_source(N=3, n=100, s=0.03, precision=precision or "fp64")
    if name == "c2":
        return checkerboard(N=7, n=280, precision=precision or "fp64")
    if name == "c3":
        return line_source(N=39, n=1000, s=0.01, precision=precision or "fp64")
    raise KeyError(name)


def gaussian_sum(s: float, centers: Sequence[tuple]) -> Field:
    """Sum of unit-mass Gaussians of standard deviation s at the given centres."""
    fs = [gaussian_std(s, cx, cy) for cx, cy in centers]

    def f(t, x, y):
        return sum(g(t, x, y) for g in fs)
    return f


def line_source_multi(N: int, n: int, s: float, centers: Sequence[tuple], half_width: float = 1.5,
                      t_final: float = 1.0, cfl: float = 0.5, precision: str = "fp64") -> Problem:
    """Line-source setting with Gaussians at several centres (corners and edges
    included), so that boundary regions carry data from the first step."""
    p = line_source(N=N, n=n, s=s, half_width=half_width, t_final=t_final, cfl=cfl, precision=precision)
    p.initial = {0: gaussian_sum(s, centers)}
    p.name = f"line_source_multi_P{N}_{n}"
    return p


def random_state(seed: int, shapes: Sequence[tuple]) -> list:
    """Seeded random moment planes (for parity tests that start from a rough state)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal(s) for s in shapes]
