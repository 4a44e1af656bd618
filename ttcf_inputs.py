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


def log_uniform_rates(count: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Shear rates drawn log-uniformly in [lo, hi] (one per start state)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))
