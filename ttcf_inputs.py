"""Seeded synthetic inputs for the TTCF path: the only module that both the GPU path's
callers and the CPU oracle's callers share.

It holds no arithmetic of the method itself: it places atoms on an fcc lattice, draws
Maxwell-Boltzmann momenta from a seeded generator, and draws per-state shear rates. The
systems are those of the paper's Example 1 (WCA fluid at the Lennard-Jones triple point,
rho = 0.8442, T = 0.722, in a cubic periodic box) at the sizes of the workloads used here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

WCA_RC = 2.0 ** (1.0 / 6.0)


@dataclass(frozen=True)
class System:
    n_cells: int           # fcc unit cells per edge; N = 4 n^3
    density: float = 0.8442
    temperature: float = 0.722
    dt: float = 0.0025

    @property
    def n(self) -> int:
        return 4 * self.n_cells ** 3

    @property
    def box(self) -> float:
        return (self.n / self.density) ** (1.0 / 3.0)

    @property
    def volume(self) -> float:
        return self.box ** 3

    @property
    def nf(self) -> int:
        """Degrees of freedom with total momentum fixed at zero."""
        return 3 * self.n - 3


def fcc_lattice(n_cells: int, box: float) -> np.ndarray:
    """fcc positions, SoA (3, N). Lattice constant a = box/n_cells, basis
    {(0,0,0), (1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2)} a shifted by (1/4,1/4,1/4) a so that no atom
    sits on a cell face. Atom order: (cx, cy, cz, basis) lexicographic."""
    a = box / n_cells
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    pos = []
    for cx in range(n_cells):
        for cy in range(n_cells):
            for cz in range(n_cells):
                for bvec in basis:
                    pos.append((np.array([cx, cy, cz], float) + bvec + 0.25) * a)
    return np.ascontiguousarray(np.array(pos).T)


def maxwell_boltzmann(n: int, temperature: float, seed: int) -> np.ndarray:
    """Momenta (3, N), unit mass: Gaussian draws from numpy's PCG64 seeded with ``seed``,
    mean removed per component, then scaled so that sum p^2 = (3N-3) T exactly."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal((3, n))
    p -= p.mean(axis=1, keepdims=True)
    p *= np.sqrt((3 * n - 3) * temperature / np.sum(p * p))
    return np.ascontiguousarray(p)


def initial_state(system: System, seed: int):
    """(r, p) SoA float64 arrays of shape (3, N) for a fresh mother."""
    return fcc_lattice(system.n_cells, system.box), maxwell_boltzmann(system.n, system.temperature, seed)


def perturbed_positions(system: System, seed: int, amplitude: float = 0.08) -> np.ndarray:
    """fcc positions with uniform random displacements of up to ``amplitude`` per component,
    wrapped into [0, L). Used for force and cell-list checks on disordered configurations."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = fcc_lattice(system.n_cells, system.box)
    r = r + rng.uniform(-amplitude, amplitude, size=r.shape)
    return np.ascontiguousarray(np.mod(r, system.box))


def ar1_series(n: int, phi: float, seed: int) -> np.ndarray:
    """A seeded first-order autoregressive series x_i = phi x_{i-1} + e_i (e_i standard
    normal, x_0 = e_0): synthetic input of known correlation for autocorrelation checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    for i in range(1, n):
        x[i] = phi * x[i - 1] + e[i]
    return x


def log_uniform_rates(count: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Shear rates drawn log-uniformly in [lo, hi] (one per start state)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))


# ----------------------------------------------------------------------------------------
# the confined channel (the paper's second example)
# ----------------------------------------------------------------------------------------

@dataclass(frozen=True)
class ChannelSystem:
    """Two walls of fcc(111) layers (triangular lattices in the x-z plane, stacked along y)
    enclosing a Lennard-Jones liquid; x and z periodic. Defaults: the full-size workload
    (2 x 3000 wall atoms in 4 layers of 25 x 30, 12000 fluid atoms at rho 0.8)."""
    n_x: int = 25               # wall atoms per row along x
    n_z: int = 30               # rows along z (even, so that the lattice is periodic)
    n_layers: int = 4
    n_fluid: int = 12000
    wall_density: float = 0.8
    fluid_density: float = 0.8
    temperature: float = 1.0    # wall thermostat target
    dt: float = 0.005
    rc: float = 2.5
    c_ff: float = 1.2
    c_wf: float = 0.6325
    k_spring: float = 150.0
    nh_tau: float = 0.5
    n_bins: int = 50

    @property
    def a_nn(self) -> float:
        """Nearest-neighbour distance of the fcc lattice of number density wall_density."""
        return (4.0 / self.wall_density) ** (1.0 / 3.0) / np.sqrt(2.0)

    @property
    def layer_gap(self) -> float:
        """Spacing of (111) planes: a / sqrt(3)."""
        return (4.0 / self.wall_density) ** (1.0 / 3.0) / np.sqrt(3.0)

    @property
    def lx(self) -> float:
        return self.n_x * self.a_nn

    @property
    def lz(self) -> float:
        return self.n_z * self.a_nn * np.sqrt(3.0) / 2.0

    @property
    def n_wall(self) -> int:
        return 2 * self.n_x * self.n_z * self.n_layers

    @property
    def n(self) -> int:
        return self.n_fluid + self.n_wall

    @property
    def gap(self) -> float:
        """Height that holds the fluid at fluid_density, plus one layer spacing for the two
        half-layers of excluded volume next to the walls; distance between the inner wall
        layers."""
        return self.n_fluid / (self.fluid_density * self.lx * self.lz) + self.layer_gap

    @property
    def y_bottom_inner(self) -> float:
        return 1.0 + (self.n_layers - 1) * self.layer_gap

    @property
    def y_top_inner(self) -> float:
        return self.y_bottom_inner + self.gap

    @property
    def y_extent(self) -> float:
        """Positions stay inside [0, y_extent)."""
        return self.y_top_inner + (self.n_layers - 1) * self.layer_gap + 1.0

    @property
    def bin_lo(self) -> float:
        return self.y_bottom_inner

    @property
    def bin_hi(self) -> float:
        return self.y_top_inner


def wall_sites(ch: ChannelSystem) -> np.ndarray:
    """Lattice sites (3, n_wall), SoA: bottom wall (outermost layer first), then top wall
    (innermost layer first). Triangular layers: row j along z at z = j a_nn sqrt(3)/2,
    x = i a_nn + (j mod 2) a_nn / 2; ABC stacking offsets 0, (a_nn/2, a_nn/(2 sqrt 3)),
    (0, a_nn/sqrt 3) in (x, z)."""
    a = ch.a_nn
    offs = [(0.0, 0.0), (0.5 * a, a / (2.0 * np.sqrt(3.0))), (0.0, a / np.sqrt(3.0))]

    def layer(y, k):
        ox, oz = offs[k % 3]
        pts = []
        for j in range(ch.n_z):
            for i in range(ch.n_x):
                x = (i * a + (j % 2) * 0.5 * a + ox) % ch.lx
                z = (j * a * np.sqrt(3.0) / 2.0 + oz) % ch.lz
                pts.append((x, y, z))
        return pts

    pts = []
    for k in range(ch.n_layers):
        pts += layer(1.0 + k * ch.layer_gap, k)
    for k in range(ch.n_layers):
        pts += layer(ch.y_top_inner + k * ch.layer_gap, ch.n_layers - 1 - k)
    return np.ascontiguousarray(np.array(pts).T)


def fluid_sites(ch: ChannelSystem) -> np.ndarray:
    """n_fluid starting positions (3, n_fluid): a simple cubic grid filling the gap (one
    spacing clear of the inner wall layers), filled row by row in (y, z, x) order."""
    ylo = ch.y_bottom_inner + 0.9
    yhi = ch.y_top_inner - 0.9
    vol = ch.lx * ch.lz * (yhi - ylo)
    s = (vol / ch.n_fluid) ** (1.0 / 3.0)
    nx = max(1, int(np.floor(ch.lx / s)))
    nz = max(1, int(np.floor(ch.lz / s)))
    ny = int(np.ceil(ch.n_fluid / (nx * nz)))
    dx, dz, dy = ch.lx / nx, ch.lz / nz, (yhi - ylo) / ny
    pts = []
    for iy in range(ny):
        for iz in range(nz):
            for ix in range(nx):
                if len(pts) < ch.n_fluid:
                    pts.append(((ix + 0.5) * dx, ylo + (iy + 0.5) * dy, (iz + 0.5) * dz))
    return np.ascontiguousarray(np.array(pts).T)


def channel_initial_state(ch: ChannelSystem, seed: int):
    """(r, p, lattice) for a fresh channel mother: fluid on its grid, wall atoms on their
    sites, Maxwell-Boltzmann momenta at the wall temperature (mean removed, scaled to
    sum p^2 = 3 N T). SoA float64 arrays (3, N) and (3, n_wall)."""
    sites = wall_sites(ch)
    r = np.concatenate([fluid_sites(ch), sites], axis=1)
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal((3, ch.n))
    p -= p.mean(axis=1, keepdims=True)
    p *= np.sqrt(3 * ch.n * ch.temperature / np.sum(p * p))
    return np.ascontiguousarray(r), np.ascontiguousarray(p), sites
