"""Seeded synthetic inputs for the slice-streaming Lennard-Jones path.

This module only *places* atoms and draws velocities; it holds none of the
method's arithmetic (no pair terms, no binning, no integration).  Both the
HIP library and the FP64 CPU oracle consume the arrays it returns, so it
imports nothing else from this package.

Workloads follow the paper's set-up (Sec. 4, first paragraph): an fcc
lattice with four atoms per lattice cell, velocities drawn for a target
temperature, reduced LJ units (sigma = epsilon = m = k_B = 1).  Where the
paper only treats N = 4*Ni^3 atoms in a cubic box, the lattice is generalised
to any N by taking the smallest lattice that covers N and removing seeded
vacancies.

Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), used as a
counter-based generator: output k of seed s is mix(s + (k+1)*gamma).
uniform = (x >> 11) * 2^-53; normals by Box-Muller with u1 = 1 - uniform.
One stream per workload is consumed in a fixed order:
vacancies -> jitter -> velocities.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = 1.0 / 9007199254740992.0

#: base seed of the named workloads; workload k uses BASE_SEED + k
BASE_SEED = 11289


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 sequence of ``seed``."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class Stream:
    """A cursor over one SplitMix64 sequence."""

    def __init__(self, seed: int):
        self.seed = int(seed)
        self.pos = 0

    def uniform(self, count: int) -> np.ndarray:
        """``count`` doubles in [0, 1)."""
        x = splitmix64(self.seed, self.pos, count)
        self.pos += count
        return (x >> np.uint64(11)).astype(np.float64) * _TWO_M53

    def normal(self, count: int) -> np.ndarray:
        """``count`` standard normals (Box-Muller, u1 = 1 - uniform in (0, 1])."""
        pairs = (count + 1) // 2
        u = self.uniform(2 * pairs)
        u1 = 1.0 - u[0::2]
        u2 = u[1::2]
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.empty(2 * pairs)
        z[0::2] = r * np.cos(2.0 * math.pi * u2)
        z[1::2] = r * np.sin(2.0 * math.pi * u2)
        return z[:count]


_FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


def fcc_counts(extent, n_atoms: int, rho: float):
    """Lattice cells per axis for ``n_atoms`` at density ``rho`` in a region of ``extent``.

    a = (4/rho)^(1/3); n_d = max(1, round(D_d / a)); while 4*nx*ny*nz < N,
    the axis with the largest D_d / n_d gets one more cell.
    """
    a = (4.0 / rho) ** (1.0 / 3.0)
    n = [max(1, int(round(d / a))) for d in extent]
    while 4 * n[0] * n[1] * n[2] < n_atoms:
        k = max(range(3), key=lambda d: extent[d] / n[d])
        n[k] += 1
    return n


def fcc_sites(origin, extent, counts) -> np.ndarray:
    """All fcc sites in (ix, iy, iz, basis) order; site = origin + (i + b + 1/4) * D/n."""
    nx, ny, nz = counts
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    frac = (cells[:, None, :] + _FCC_BASIS[None, :, :] + 0.25).reshape(-1, 3)
    step = np.array([extent[0] / nx, extent[1] / ny, extent[2] / nz])
    return np.asarray(origin, dtype=np.float64) + frac * step


def remove_vacancies(sites: np.ndarray, n_keep: int, stream: Stream) -> np.ndarray:
    """Seeded partial Fisher-Yates: drop len(sites) - n_keep sites, keep the order."""
    m = len(sites) - n_keep
    if m <= 0:
        return sites
    total = len(sites)
    idx = np.arange(total, dtype=np.int64)
    u = stream.uniform(m)
    for k in range(m):
        j = k + int(u[k] * (total - k))
        idx[k], idx[j] = idx[j], idx[k]
    keep = np.ones(total, dtype=bool)
    keep[idx[:m]] = False
    return sites[keep]


def _wrap(pos: np.ndarray, box) -> None:
    for d in range(3):
        col = pos[:, d]
        col[col >= box[d]] -= box[d]
        col[col < 0.0] += box[d]


def jitter(pos: np.ndarray, box, stream: Stream, amp: float = 0.05) -> None:
    """Each coordinate += U[-amp, amp), then wrap into the box (in place)."""
    u = stream.uniform(pos.size).reshape(pos.shape)
    pos += (2.0 * amp) * u - amp
    _wrap(pos, box)


def maxwell_boltzmann(n: int, T: float, stream: Stream) -> np.ndarray:
    """N(0, T) per component, mean removed, rescaled to T_inst = T with 3N-3 dof (m = 1)."""
    v = stream.normal(3 * n).reshape(n, 3) * math.sqrt(T)
    if n <= 1:
        return np.zeros((n, 3))
    v -= v.mean(axis=0)
    ke2 = float(np.sum(v * v))  # 2K
    t_inst = ke2 / (3 * n - 3)
    if t_inst > 0.0:
        v *= math.sqrt(T / t_inst)
    return v


@dataclass
class System:
    """One synthetic LJ system: box, slices and the id-ordered state."""

    name: str
    box: tuple
    slices: int
    pos: np.ndarray
    vel: np.ndarray
    rc: float = 2.5
    dt: float = 0.005
    steps: int = 100
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.pos)


def homogeneous(n: int, rho: float, T: float, seed: int, aspect=(1.0, 1.0, 1.0)):
    """Homogeneous fluid in a periodic box with edge ratios ``aspect`` (volume n/rho)."""
    vol = n / rho
    unit = (vol / (aspect[0] * aspect[1] * aspect[2])) ** (1.0 / 3.0)
    box = tuple(float(unit * a) for a in aspect)
    st = Stream(seed)
    counts = fcc_counts(box, n, rho)
    sites = fcc_sites((0.0, 0.0, 0.0), box, counts)
    pos = np.ascontiguousarray(remove_vacancies(sites, n, st))
    jitter(pos, box, st)
    vel = np.ascontiguousarray(maxwell_boltzmann(n, T, st))
    return box, pos, vel, {"fcc": counts, "vacancies": 4 * counts[0] * counts[1] * counts[2] - n,
                           "rho": rho, "T": T}


def slab(n: int, rho_l: float, rho_v: float, T: float, seed: int, elong: float = 16.0):
    """Vapour-liquid slab: liquid in x in [Lx/3, 2Lx/3), vapour in the rest (one periodic region).

    Lx = elong * Ly, Ly = Lz.  The volume follows from n = rho_l V/3 + rho_v 2V/3;
    N_liquid = round(rho_l V/3), the vapour takes the remainder.  Liquid atoms come
    first in id order.
    """
    vol = n / (rho_l / 3.0 + 2.0 * rho_v / 3.0)
    ly = (vol / elong) ** (1.0 / 3.0)
    box = (elong * ly, ly, ly)
    n_l = int(round(rho_l * vol / 3.0))
    n_v = n - n_l
    st = Stream(seed)
    ext_l = (box[0] / 3.0, ly, ly)
    ext_v = (2.0 * box[0] / 3.0, ly, ly)
    c_l = fcc_counts(ext_l, n_l, rho_l)
    c_v = fcc_counts(ext_v, n_v, rho_v)
    s_l = remove_vacancies(fcc_sites((box[0] / 3.0, 0.0, 0.0), ext_l, c_l), n_l, st)
    s_v = remove_vacancies(fcc_sites((2.0 * box[0] / 3.0, 0.0, 0.0), ext_v, c_v), n_v, st)
    pos = np.ascontiguousarray(np.concatenate([s_l, s_v]))
    _wrap(pos, box)
    jitter(pos, box, st)
    vel = np.ascontiguousarray(maxwell_boltzmann(n, T, st))
    meta = {"n_liquid": n_l, "n_vapour": n_v, "fcc_liquid": c_l, "fcc_vapour": c_v,
            "rho": [rho_l, rho_v], "T": T,
            "vacancies_liquid": 4 * c_l[0] * c_l[1] * c_l[2] - n_l,
            "vacancies_vapour": 4 * c_v[0] * c_v[1] * c_v[2] - n_v}
    return box, pos, vel, meta


# ---------------------------------------------------------------------------
# Named workloads (the paper's homogeneous fcc LJ fluid at the sizes studied here)
# ---------------------------------------------------------------------------

def lj_fluid_2048(seed: int = BASE_SEED + 0) -> System:
    """N=2048 at rho=0.8, T=1.0, cubic, 4 x-slices, 100 steps (CPU-checkable)."""
    box, pos, vel, meta = homogeneous(2048, 0.8, 1.0, seed)
    return System("lj_fluid_2048", box, 4, pos, vel, steps=100, meta=meta)


def lj_fluid_4m(seed: int = BASE_SEED + 1) -> System:
    """N=4,194,304 at rho=0.8, T=1.0, cubic, 64 x-slices, 1000 steps."""
    box, pos, vel, meta = homogeneous(4194304, 0.8, 1.0, seed)
    return System("lj_fluid_4m", box, 64, pos, vel, steps=1000, meta=meta)


def lj_liquid_32m(seed: int = BASE_SEED + 2) -> System:
    """N=33,554,432 near the triple point (rho=0.85, T=0.9), 4:1:1 box, 256 x-slices."""
    box, pos, vel, meta = homogeneous(33554432, 0.85, 0.9, seed, aspect=(4.0, 1.0, 1.0))
    return System("lj_liquid_32m", box, 256, pos, vel, steps=1000, meta=meta)


def lj_slab_8m(seed: int = BASE_SEED + 3) -> System:
    """N=8,388,608 vapour-liquid slab (rho_l=0.73, rho_v=0.02, T=0.8), Lx=16Ly, 512 x-slices."""
    box, pos, vel, meta = slab(8388608, 0.73, 0.02, 0.8, seed)
    return System("lj_slab_8m", box, 512, pos, vel, steps=2000, meta=meta)


@dataclass
class Request:
    """One served run: arrival time (s) and its state point."""

    index: int
    arrival: float
    n: int
    rho: float
    T: float
    steps: int
    seed: int

    def system(self) -> System:
        box, pos, vel, meta = homogeneous(self.n, self.rho, self.T, self.seed)
        slices = int(math.floor(box[0] / 2.5))
        return System(f"served_{self.index}", box, slices, pos, vel, steps=self.steps, meta=meta)


def served_ensemble(count: int = 2000, rate: float = 50.0, seed: int = BASE_SEED + 4):
    """Poisson arrivals at ``rate``/s; N log-uniform [500, 2e5], rho U[0.3, 0.9],
    T U[0.8, 2.0], steps uniform in {200..2000}.  Request k's own state is drawn from
    seed + k (after the schedule stream)."""
    st = Stream(seed)
    u = st.uniform(5 * count).reshape(count, 5)
    t = 0.0
    out = []
    for k in range(count):
        t += -math.log(1.0 - u[k, 0]) / rate
        n = int(round(math.exp(math.log(500.0) + u[k, 1] * (math.log(2.0e5) - math.log(500.0)))))
        rho = 0.3 + 0.6 * u[k, 2]
        T = 0.8 + 1.2 * u[k, 3]
        steps = 200 + int(u[k, 4] * 1801)
        out.append(Request(k, t, n, rho, T, steps, seed + 1 + k))
    return out


WORKLOADS = {
    "lj_fluid_2048": lj_fluid_2048,
    "lj_fluid_4m": lj_fluid_4m,
    "lj_liquid_32m": lj_liquid_32m,
    "lj_slab_8m": lj_slab_8m,
}
