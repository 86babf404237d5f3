"""Seeded diagonal phonon self-energies (inputs only, no method arithmetic).

Section 1 includes a phonon self-energy in A and takes it diagonal: one
complex value per site and energy.  These generators give it the shape of
local elastic dephasing with a local occupation (a Buttiker-probe-like
model): per site k and energy E

  Sigma^r_ph(k, E) = delta_k - i gamma_k(E) / 2,
  Sigma^<_ph(k, E) = i gamma_k(E) f(E; mu_k, kT),

with gamma_k(E) = gamma0 (1 + spread r_k) (1 + 0.2 sin(E / 0.05 + phi_k)),
r_k uniform in [-1/2, 1/2], delta_k uniform in [-gamma0/4, gamma0/4], phi_k
uniform in [0, 2 pi), and mu_k interpolated linearly between the two contact
levels along the transport coordinate (equilibrium=True: one level
mu_k = mu[0] everywhere, the fluctuation-dissipation case
Sigma^< = -f (Sigma^r - Sigma^r+)).  Sigma^<_ph is anti-Hermitian (purely
imaginary on the diagonal) and Im Sigma^r_ph < 0, as for the contacts.
"""
from __future__ import annotations

import numpy as np

from . import leads


def transport_fraction(device) -> np.ndarray:
    """Position of every site along the transport direction, scaled to
    [0, 1]: the first coordinate when the device has coordinates, else the
    site index."""
    if getattr(device, "coords", None) is not None:
        x = np.asarray(device.coords, dtype=np.float64).reshape(device.n, -1)[:, 0]
    else:
        x = np.arange(device.n, dtype=np.float64)
    span = x.max() - x.min()
    return (x - x.min()) / span if span > 0 else np.zeros_like(x)


def diagonal_self_energies(device, energies, gamma0: float = 5e-3, mu=(0.10, 0.05),
                           kt: float = 0.025, spread: float = 0.5, seed: int = 0,
                           equilibrium: bool = False):
    """(sig_r_ph, sig_less_ph), each complex128 [nE, n] in the device's site
    order."""
    rng = np.random.default_rng(seed)
    n = device.n
    e = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    r = rng.uniform(-0.5, 0.5, n)
    delta = rng.uniform(-0.25, 0.25, n) * gamma0
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    gam = gamma0 * (1.0 + spread * r)[None, :] * (1.0 + 0.2 * np.sin(e[:, None] / 0.05 + phi[None, :]))
    if equilibrium:
        mu_k = np.full(n, float(mu[0]))
    else:
        x = transport_fraction(device)
        mu_k = float(mu[0]) + (float(mu[1]) - float(mu[0])) * x
    f = leads.fermi(e[:, None] - mu_k[None, :], 0.0, kt)
    sig_r = delta[None, :] - 0.5j * gam
    sig_l = 1j * gam * f
    return sig_r.astype(np.complex128), sig_l.astype(np.complex128)
