"""Seeded synthetic initial states, shared by the engine's tests, the benchmark
and the oracle checks.

This module only draws random numbers and lays out a lattice: it contains none
of the method's arithmetic (no distances, no forces, no integration).  The
paper simulates self-generated fluids (Models section: LJ and patchy systems at
given number density and temperature); these states stand in for them.

Recipe (fixed draw order, numpy PCG64 ``default_rng(seed + 1000 * attempt)``):
  1. simple-cubic lattice with n = ceil(N^(1/3)) sites per side and spacing
     L/n, sites at (k + 1/2) * L/n, the first N sites in x-fastest order;
  2. jitter U[-0.05, 0.05] sigma per component, then wrapped into [0, L);
  3. velocities N(0, sqrt(T/m)) per component, mean removed, rescaled so that
     sum m v^2 / (3N - 3) = T exactly;
  4. patchy only: quaternions from 4 standard normals, normalised (uniform on
     SO(3)); angular momenta N(0, sqrt(I T)) per component.
``attempt`` lets a caller redraw the jitter when a state is rejected (e.g.
because a pair distance sits within 1e-9 sigma of a cut-off).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    pot: str                # "lj" or "patchy"
    n: int
    rho: float
    temp: float
    rcut: float
    skin: float = 0.3
    dt: float = 0.001
    steps: int = 100
    eps: float = 1.0
    sigma: float = 1.0
    mass: float = 1.0
    # patchy only
    eps_p: float = 1.0
    patch_w: float = 0.12
    patch_delta: float = 0.5
    patch_rcut: float = 0.75
    inertia: float = 1.0
    patch_model: str = "tetra"  # "tetra" (four patches) or "polar2" (the paper's two)
    max_neighbors: int = 0  # 0: choose from the density

    @property
    def box(self) -> float:
        return (self.n / self.rho) ** (1.0 / 3.0)

    @property
    def rv(self) -> float:
        return self.rcut + self.skin

    def expected_neighbors(self) -> float:
        """Mean full-list length of a uniform fluid, rho * 4/3 pi r_v^3."""
        return self.rho * 4.0 / 3.0 * math.pi * self.rv ** 3

    def list_capacity(self) -> int:
        if self.max_neighbors:
            return self.max_neighbors
        m = self.expected_neighbors()
        # uniform-fluid mean plus a wide margin for fluctuations; multiple of 16
        cap = int(math.ceil((1.5 * m + 8 * math.sqrt(m) + 16) / 16.0) * 16)
        return cap

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The systems studied (densities, temperatures and cut-offs of the LJ and
# patchy fluids; see the workload recipe in the design notes).
WORKLOADS = {
    "lj_small": Workload("lj_small", "lj", 4096, 0.8, 1.5, 2.5, steps=100),
    "lj_many": Workload("lj_many", "lj", 262144, 0.8, 1.5, 2.5, steps=1000),
    "lj_many_dense": Workload("lj_many_dense", "lj", 262144, 1.0, 1.5, 3.0, steps=1000),
    "patchy": Workload("patchy", "patchy", 131072, 0.5, 0.2, 1.5, steps=1000),
    # the paper's patchy model: two polar patches, (sigma/r)^200 core, patch
    # range 0.18 sigma, so r_c = 2 delta + 0.18 = 1.18; k_B T / eps = 0.15
    "patchy_paper": Workload("patchy_paper", "patchy", 131072, 0.5, 0.15, 1.18, steps=1000,
                             patch_rcut=0.18, patch_model="polar2"),
    "lj_precision": Workload("lj_precision", "lj", 1048576, 0.8, 1.0, 2.5, dt=0.005,
                             steps=10000),
}


@dataclass
class State:
    x: np.ndarray          # (N, 3) float64 positions in [0, L)
    v: np.ndarray          # (N, 3) float64 velocities
    q: np.ndarray | None   # (N, 4) float64 unit quaternions (w, x, y, z), patchy
    angmom: np.ndarray | None  # (N, 3) float64 angular momenta, patchy
    box: float
    seed: int
    attempt: int


def lattice(n: int, box: float) -> np.ndarray:
    m = int(math.ceil(round(n ** (1.0 / 3.0), 12)))
    while m ** 3 < n:
        m += 1
    a = box / m
    k = np.arange(n)
    ix, iy, iz = k % m, (k // m) % m, k // (m * m)
    return (np.stack([ix, iy, iz], axis=1).astype(np.float64) + 0.5) * a


def chain_columns(n: int, box: float, bond: float = 1.04):
    """Sites on columns along z: each column holds nz = floor(box / bond)
    sites spaced box / nz (>= bond), the columns sit on a square grid in
    (x, y) filled one column at a time."""
    nz = max(int(box // bond), 1)
    ncol = -(-n // nz)
    m = int(math.ceil(math.sqrt(ncol)))
    a, b = box / m, box / nz
    k = np.arange(n)
    c, iz = k // nz, k % nz
    return np.stack([(c % m + 0.5) * a, (c // m + 0.5) * a, (iz + 0.5) * b], axis=1)


def make_state(w: Workload, seed: int, attempt: int = 0) -> State:
    rng = np.random.default_rng(seed + 1000 * attempt)
    L = w.box
    n = w.n
    if w.patch_model == "polar2":
        # chains along z with the patch axes mostly along the chain, so that
        # about half the neighbouring patches are bonded (a stand-in for the
        # chain fluid the two-patch model forms at k_B T = 0.15)
        x = chain_columns(n, L) + rng.uniform(-0.02, 0.02, size=(n, 3)) * w.sigma
    else:
        x = lattice(n, L) + rng.uniform(-0.05, 0.05, size=(n, 3)) * w.sigma
    x = np.mod(x, L)
    x[x >= L] -= L
    v = rng.normal(0.0, math.sqrt(w.temp / w.mass), size=(n, 3))
    v -= v.mean(axis=0)
    dof = 3 * n - 3
    t_now = (w.mass * (v * v).sum()) / dof
    v *= math.sqrt(w.temp / t_now)
    q = am = None
    if w.pot == "patchy":
        q = rng.normal(size=(n, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        am = rng.normal(0.0, math.sqrt(w.inertia * w.temp), size=(n, 3))
        if w.patch_model == "polar2":
            # 70 %: body z along the lab z axis, tilted by an angle N(0, 0.15)
            # about a random axis in the xy plane: q = (cos h, sin h ax, sin h ay, 0)
            aligned = rng.random(n) < 0.7
            h = 0.5 * rng.normal(0.0, 0.15, size=n)
            phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
            qa = np.stack([np.cos(h), np.sin(h) * np.cos(phi), np.sin(h) * np.sin(phi),
                           np.zeros(n)], axis=1)
            q[aligned] = qa[aligned]
    return State(x=x, v=v, q=q, angmom=am, box=L, seed=seed, attempt=attempt)


@dataclass(frozen=True)
class Request:
    """One serving request: simulate `workload` (its n, potential, density and
    step count) from make_state(workload, seed)."""
    rid: int
    arrival: float  # seconds after the stream starts
    workload: Workload
    seed: int


def serving_requests(count: int, rate_hz: float, seed: int = 0, steps: int = 1000,
                     n_min: int = 500, n_max: int = 50000,
                     patchy_share: float = 0.3) -> list[Request]:
    """A stream of independent simulation requests.

    Recipe (numpy PCG64 ``default_rng(seed)``, four draws per request in this
    order): exponential inter-arrival gap of mean 1/rate_hz (Poisson
    arrivals); log N uniform in [log n_min, log n_max], rounded; patchy with
    probability patchy_share, else LJ; density U[0.3, 0.6] for patchy and
    U[0.6, 0.9] for LJ.  The LJ and patchy requests otherwise take the
    parameters of the lj_small and patchy workloads (cut-offs, temperature,
    skin, dt).  Request k's state seed is 1 + k.
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for k in range(count):
        t += rng.exponential(1.0 / rate_hz)
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        patchy = rng.random() < patchy_share
        rho = rng.uniform(0.3, 0.6) if patchy else rng.uniform(0.6, 0.9)
        base = WORKLOADS["patchy" if patchy else "lj_small"]
        w = base.with_(name=f"req{k}", n=n, rho=float(rho), steps=steps)
        out.append(Request(rid=k, arrival=t, workload=w, seed=1 + k))
    return out
