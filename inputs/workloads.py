"""The synthetic workloads (shapes of Section 4.2's superlattice and carbon
tube experiments), each fully determined by its seed.

Each builder returns a Workload: a Device, the energy grid, the broadening
eta, the contact chemical potentials, kT, and quadrature weights c_E for the
density n_i = sum_E c_E (-i G^<_ii(E)).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import devices, leads


@dataclasses.dataclass
class Workload:
    name: str
    device: devices.Device
    energies: np.ndarray
    eta: float
    mu: tuple
    kt: float
    potential: np.ndarray | None = None   # on-site V (added to diag H), separate input

    def quad_weights(self) -> np.ndarray:
        """Trapezoid weights c_E = w_E dE / (2 pi) on the (uniform) energy grid."""
        e = self.energies
        if e.size < 2:
            return np.ones_like(e) / (2 * np.pi)
        w = np.full(e.size, e[1] - e[0])
        w[0] *= 0.5
        w[-1] *= 0.5
        return w / (2 * np.pi)

    def self_energies(self, energies=None):
        e = self.energies if energies is None else np.asarray(energies)
        return leads.contact_self_energies(self.device, e, self.eta, self.mu, self.kt)


def uniform_waveguide(n_transport=64, n_transverse=32, n_energies=16, emax=0.3, eta=1e-6,
                      mu=(0.10, 0.05), kt=0.025) -> Workload:
    """Uniform hard-wall waveguide (V = 0): 64 x 32 grid, a = 0.25 nm,
    m* = 0.067, 16 energies in [0, 0.3] eV."""
    dev = devices.fd2d(n_transport, n_transverse, 0.25, 0.067, name="waveguide")
    return Workload("waveguide_%dx%d" % (n_transport, n_transverse), dev,
                    np.linspace(0.0, emax, n_energies), eta, mu, kt)


def superlattice(n_transport=1024, n_transverse=64, n_energies=512, eta=1e-6, mu=(0.10, 0.05),
                 kt=0.025, seed=2) -> Workload:
    """Quantum-well superlattice on a 1024 x 64 grid: 20-layer flat ends,
    repeating 20-layer (5 nm) wells and 8-layer (2 nm) 0.3 eV barriers,
    +-10 meV seeded on-site noise, 512 energies in [0, 0.5] eV."""
    v = devices.superlattice_potential(n_transport, n_transverse, seed=seed)
    dev = devices.fd2d(n_transport, n_transverse, 0.25, 0.067, potential=v,
                       name="superlattice")
    return Workload("superlattice_%dx%d" % (n_transport, n_transverse), dev,
                    np.linspace(0.0, 0.5, n_energies), eta, mu, kt)


def uneven_devices(n_devices=64, n_energies=128, eta=1e-6, mu=(0.10, 0.05), kt=0.025,
                   widths=(32, 48, 64, 96, 128), lmin=256, lmax=2048, base_seed=3000):
    """Batch of 2-D FD devices of uneven widths and lengths with random
    barrier profiles, 128 energies each in [0, 0.5] eV."""
    return [uneven_device(d, n_energies, eta, mu, kt, widths, lmin, lmax, base_seed)
            for d in range(n_devices)]


def uneven_device(d, n_energies=128, eta=1e-6, mu=(0.10, 0.05), kt=0.025,
                  widths=(32, 48, 64, 96, 128), lmin=256, lmax=2048, base_seed=3000) -> Workload:
    """Device d of the uneven batch (seed base_seed + d)."""
    rng = np.random.default_rng(base_seed + d)
    w = int(rng.choice(widths))
    l = int(rng.integers(lmin, lmax + 1))
    v = devices.barrier_potential(l, w, rng)
    dev = devices.fd2d(l, w, 0.25, 0.067, potential=v, name="device%d" % d)
    return Workload("uneven%d_%dx%d" % (d, l, w), dev, np.linspace(0.0, 0.5, n_energies), eta,
                    mu, kt)


def nanotube(n_cells=2000, n_energies=256, eta=1e-6, mu=(0.05, -0.05), kt=0.025,
             seed=4) -> Workload:
    """(10,0) zigzag tube, nearest-neighbour t = -2.7 eV, 2000 cells of 40
    atoms (80 000 orbitals), Anderson disorder +-0.2 eV, 256 energies in
    [-1, 1] eV."""
    dev = devices.zigzag_tube(n_cells, 10, -2.7, 0.2, seed)
    return Workload("tube10_%dcells" % n_cells, dev, np.linspace(-1.0, 1.0, n_energies),
                    eta, mu, kt)


def armchair_ribbon(n_cells=60, n_lines=7, n_energies=6, emin=-1.2, emax=1.2, eta=1e-6,
                    mu=(0.05, -0.05), kt=0.025, disorder=0.2, vacancies=0.03, seed=6) -> Workload:
    """Armchair graphene nanoribbon (7 dimer lines, 14 atoms per cell),
    t = -2.7 eV, Anderson disorder and seeded vacancies: the honeycomb
    stencil on an irregular graph."""
    dev = devices.armchair_ribbon(n_cells, n_lines, -2.7, disorder, vacancies, seed)
    return Workload("agnr%d_%dcells" % (n_lines, n_cells), dev, np.linspace(emin, emax, n_energies),
                    eta, mu, kt)


def adjoint_device(n_transport=512, n_transverse=64, n_energies=256, eta=1e-6, mu=(0.10, 0.05),
                   kt=0.025, seed=5) -> Workload:
    """512 x 64 grid with a seeded smooth random potential (max |V| = 50 meV)
    supplied separately as the differentiable input V; 256 energies in
    [0, 0.5] eV."""
    dev = devices.fd2d(n_transport, n_transverse, 0.25, 0.067, name="adjoint")
    v = devices.smooth_random_potential(n_transport, n_transverse, 0.050, 8.0, seed)
    return Workload("adjoint_%dx%d" % (n_transport, n_transverse), dev,
                    np.linspace(0.0, 0.5, n_energies), eta, mu, kt, potential=v)


def small_grid(n_transport, n_transverse, n_energies=4, emin=0.0, emax=0.3, eta=1e-3,
               mu=(0.10, 0.05), kt=0.025, noise=0.0, seed=0) -> Workload:
    """Small FD grid used by parity tests (optionally with seeded noise)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-noise, noise, n_transport * n_transverse) if noise > 0 else None
    dev = devices.fd2d(n_transport, n_transverse, 0.25, 0.067, potential=v, name="small")
    return Workload("small_%dx%d" % (n_transport, n_transverse), dev,
                    np.linspace(emin, emax, n_energies), eta, mu, kt)
