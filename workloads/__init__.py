"""Seeded synthetic inputs shaped like the paper's workloads.

This module only produces inputs (potentials, disorder draws, initial wave
packets, system lists).  It holds none of the propagation method's
arithmetic, and both the GPU library's tests and the CPU oracle's tests draw
their inputs from here.

Workload shapes follow Fehske et al., arXiv:0907.3022: the 1D double well and
Gaussian packet eq. (psi0) of Sect. 3.1, the disordered honeycomb ribbon of
eq. (model) (Sect. 3.2), and the Holstein polaron of eq. (ghm) (Sect. 3.3).

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), mapped to doubles in [0, 1)
as (u >> 11) * 2^-53.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """First `count` outputs of SplitMix64 seeded with `seed` (uint64 array)."""
    with np.errstate(over="ignore"):
        idx = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) from SplitMix64: (u >> 11) * 2^-53."""
    u = splitmix64(seed, count)
    return (u >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# --------------------------------------------------------------------------
# 1D grid, potentials and packets (Sect. 3.1)
# --------------------------------------------------------------------------
def chain_grid(n: int, xmin: float = -20.0, xmax: float = 20.0):
    """n equally spaced points on [xmin, xmax]; returns (x, dx)."""
    dx = (xmax - xmin) / (n - 1)
    x = xmin + dx * np.arange(n, dtype=np.float64)
    return x, dx


def quartic_well(x: np.ndarray, a: float = 0.05, b: float = 5.0) -> np.ndarray:
    """V(x) = a (x^2 - b^2)^2: symmetric double well, minima at +-b."""
    return a * (x * x - b * b) ** 2


def paper_double_well(x: np.ndarray, omega0: float = 0.4, aq: float = 0.02,
                      V0: float = 1.0, m: float = 1.0) -> np.ndarray:
    """V(q) = V0 + (1/2) m omega0^2 (-q^2 + a q^4) with the Sect. 3.1 values."""
    return V0 + 0.5 * m * omega0 ** 2 * (-x * x + aq * x ** 4)


def harmonic(x: np.ndarray, omega: float) -> np.ndarray:
    return 0.5 * omega * omega * x * x


def gaussian_1d(x: np.ndarray, x0: float, sigma: float, k0: float) -> np.ndarray:
    """Packet of eq. (psi0): exp(-(x-x0)^2/(4 sigma^2) + i k0 x), unit 2-norm."""
    psi = np.exp(-((x - x0) ** 2) / (4.0 * sigma * sigma) + 1j * k0 * x)
    return (psi / np.linalg.norm(psi)).astype(np.complex128)


# --------------------------------------------------------------------------
# honeycomb ribbons (Sect. 3.2, eq. (model)); site index y*length + x
# --------------------------------------------------------------------------
def anderson_disorder(width: int, length: int, W: float, seed: int) -> np.ndarray:
    """On-site energies eps_j uniform in [-W/2, W/2), one SplitMix64 draw per site."""
    return W * (uniform01(seed, width * length) - 0.5)


def gaussian_ribbon(width: int, length: int, x0: float, y0: float, sigma: float,
                    k0: float) -> np.ndarray:
    """exp(-((x-x0)^2+(y-y0)^2)/(4 sigma^2) + i k0 x) on the grid, unit 2-norm."""
    y, x = np.meshgrid(np.arange(width, dtype=np.float64),
                       np.arange(length, dtype=np.float64), indexing="ij")
    psi = np.exp(-((x - x0) ** 2 + (y - y0) ** 2) / (4.0 * sigma * sigma) + 1j * k0 * x)
    psi = psi.reshape(-1)
    return (psi / np.linalg.norm(psi)).astype(np.complex128)


def ribbon_packet(width: int, length: int, sigma: float = 20.0, k0: float = 1.0) -> np.ndarray:
    """Injected packet: centred at x0 = length/4, y0 = (width-1)/2."""
    return gaussian_ribbon(width, length, length / 4.0, (width - 1) / 2.0, sigma, k0)


def single_site(n: int, i: int) -> np.ndarray:
    psi = np.zeros(n, dtype=np.complex128)
    psi[i] = 1.0
    return psi


def random_state(n: int, seed: int) -> np.ndarray:
    """Dense complex vector with unit 2-norm: real and imaginary parts uniform
    in [-1/2, 1/2) from one SplitMix64 stream (re, im of site i from outputs
    2i and 2i+1).  Every site carries an amplitude of order 1/sqrt(n)."""
    u = uniform01(seed, 2 * n) - 0.5
    psi = u[0::2] + 1j * u[1::2]
    return (psi / np.linalg.norm(psi)).astype(np.complex128)


def random_weights(n: int, seed: int) -> np.ndarray:
    """Dense real weights in [0, 1) from SplitMix64 (a loss sum_i w_i |psi_i|^2
    then has a nonzero adjoint on every site)."""
    return uniform01(seed, n)


def right_half_mask_ribbon(width: int, length: int) -> np.ndarray:
    """1 where the column lies right of the ribbon centre (x > (length-1)/2)."""
    x = np.tile(np.arange(length), width)
    return (x > (length - 1) / 2.0).astype(np.float64)


# --------------------------------------------------------------------------
# Holstein polaron (Sect. 3.3, eq. (ghm))
# --------------------------------------------------------------------------
def holstein_vacuum_site(L: int, site: int, nconf: int) -> np.ndarray:
    """Bare electron at `site` with no phonons: state index site * nconf + rank,
    and the phonon vacuum has rank 0."""
    return single_site(nconf * L, site * nconf)


def holstein_packet(L: int, nconf: int, centre: float, width: float, k: float) -> np.ndarray:
    """Bare-electron Gaussian packet exp(-(i-c)^2/(4 w^2) + i k i) times phonon vacuum."""
    i = np.arange(L, dtype=np.float64)
    e = np.exp(-((i - centre) ** 2) / (4.0 * width * width) + 1j * k * i)
    e /= np.linalg.norm(e)
    psi = np.zeros(nconf * L, dtype=np.complex128)
    psi[::nconf] = e  # rank 0 (vacuum) of every site
    return psi


# --------------------------------------------------------------------------
# batched disorder realisations
# --------------------------------------------------------------------------
@dataclass
class RibbonSystem:
    width: int
    length: int
    W: float
    seed: int

    @property
    def n(self) -> int:
        return self.width * self.length


def batched_ribbons(nsys: int = 256, seed_base: int = 1000, wmin: int = 32, wmax: int = 128,
                    lmin: int = 512, lmax: int = 4096, Wlo: float = 0.1, Whi: float = 2.0):
    """nsys ribbons with width U{wmin..wmax}, length U{lmin..lmax}, W U[Wlo, Whi];
    system s draws its disorder with seed seed_base + s."""
    u = uniform01(seed_base ^ 0x5EEDBA7C4, 3 * nsys).reshape(nsys, 3)
    out = []
    for s in range(nsys):
        w = wmin + int(u[s, 0] * (wmax - wmin + 1))
        l = lmin + int(u[s, 1] * (lmax - lmin + 1))
        W = Wlo + (Whi - Wlo) * u[s, 2]
        out.append(RibbonSystem(w, l, W, seed_base + s))
    return out


# --------------------------------------------------------------------------
# the five workload presets
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    params: dict = field(default_factory=dict)


DOUBLE_WELL = Workload("double_well_1d", dict(n=4096, xmin=-20.0, xmax=20.0, a=0.05, b=5.0,
                                               x0=-5.0, sigma=1.0, k0=1.0, dt=0.5, K=200))
GRAPHENE = Workload("zigzag_ribbon_128x8192", dict(width=128, length=8192, edge="zigzag", t=1.0,
                                                   W=0.5, seed=0, sigma=20.0, k0=1.0, dt=1.0,
                                                   K=1000))
HOLSTEIN = Workload("holstein_ring_L10_nph10", dict(L=10, nph=10, t=1.0, w0=1.0, g2=(0.5, 2.0),
                                                    periodic=True, dt=0.1, K=500))
BATCHED = Workload("batched_256_ribbons", dict(nsys=256, seed_base=1000, dt=1.0, K=200))
# Sect. 3.3 / Fig. 3: open 18-site chain, at most 11 phonons (D = 622,751,220),
# eps_p = 1, w0 = 2 (g = sqrt(eps_p / w0)), barrier Delta = 2 at site 12 with an
# extra local coupling eps_p,12 there, packet around site 4 moving with k = pi/9.
# Not printed, chosen here: eps_p,12 = eps_p, packet width 2 sites, dt = 0.5.
POLARON_PAPER = Workload("polaron_L18_nph11", dict(L=18, nph=11, t=1.0, w0=2.0, eps_p=1.0,
                                                   eps_p_barrier=1.0, barrier_site=11,
                                                   barrier=2.0, packet_site=3, k=math.pi / 9,
                                                   width=2.0, dt=0.5, snapshots=(6.0, 10.0, 14.0)))
# Sect. 3.2 / Table 2: armchair ribbon of 10 x 1000 atoms, one occupied site
# at the centre, propagated to t = 1e4 with dt = 1, 10, 100.  Not printed for
# the timings, chosen here: disorder W = 0.5 (the weakest of Fig. 2), seed 2.
TABLE2 = Workload("armchair_ribbon_10x1000_t1e4", dict(width=10, length=1000, edge="armchair", t=1.0,
                                                       W=0.5, seed=2, t_end=1e4, dts=(1.0, 10.0, 100.0)))
ADJOINT = Workload("adjoint_transmission", dict(n1d=65536, width=256, length=4096, W=0.5, K=100,
                                                order=64, fd_sites=32, h=1e-6))


def ribbon_inputs(width: int, length: int, W: float, seed: int, sigma: float = 20.0,
                  k0: float = 1.0):
    """(eps, psi0) for one disordered ribbon with the injected packet."""
    eps = anderson_disorder(width, length, W, seed)
    sig = min(sigma, width / 4.0)
    psi = ribbon_packet(width, length, sig, k0)
    return eps, psi


def table2_inputs(width: int, length: int, W: float, seed: int):
    """(eps, psi0) for the Table 2 ribbon: disorder and the single site at the
    centre (row width // 2, column length // 2)."""
    eps = anderson_disorder(width, length, W, seed)
    return eps, single_site(width * length, (width // 2) * length + length // 2)


def double_well_inputs(n: int = 4096, xmin: float = -20.0, xmax: float = 20.0, a: float = 0.05,
                       b: float = 5.0, x0: float = -5.0, sigma: float = 1.0, k0: float = 1.0):
    x, dx = chain_grid(n, xmin, xmax)
    return x, dx, quartic_well(x, a, b), gaussian_1d(x, x0, sigma, k0)


def polaron_couplings(L: int, w0: float, eps_p: float, eps_p_barrier: float, barrier_site: int,
                      barrier: float):
    """(g_i, Delta_i) of eq. (ghm): g_i = sqrt((eps_p + eps_p,i)/w0), with the
    extra coupling and the barrier potential only on `barrier_site`."""
    extra = np.zeros(L)
    extra[barrier_site] = eps_p_barrier
    g = np.sqrt((eps_p + extra) / w0)
    Delta = np.zeros(L)
    Delta[barrier_site] = barrier
    return g, Delta


def fd_sites(n: int, count: int, seed: int, candidates=None) -> np.ndarray:
    """`count` distinct seeded site indices (from `candidates` if given)."""
    pool = np.arange(n) if candidates is None else np.asarray(candidates)
    u = uniform01(seed, 4 * count + 16)
    picked = []
    for v in u:
        j = int(pool[int(v * pool.size)])
        if j not in picked:
            picked.append(j)
        if len(picked) == count:
            break
    return np.array(sorted(picked), dtype=np.int64)


def comb(n: int, k: int) -> int:
    return math.comb(n, k)
