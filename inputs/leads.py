"""Contact self-energies of semi-infinite leads, and lesser self-energies.

Section 2: the semi-infinite leads are folded into the first and last layer
as dense blocks Sigma^r_L, Sigma^r_R.  Section 3 assumes Sigma^< block
diagonal, skew-Hermitian and purely imaginary; for a contact in equilibrium
at Fermi level mu, Sigma^< = i f(E) Gamma with Gamma = i (Sigma^r - Sigma^r+).

Two independent constructions:
  * fd_lead_sigma: the hard-wall effective-mass lead, diagonal in the
    transverse sine modes, each mode a 1-D chain whose surface Green's
    function has a closed form;
  * sancho_rubio: the decimation of Lopez Sancho, Lopez Sancho and Rubio
    (J. Phys. F 15, 851 (1985)) for any lead given by cell blocks H00, H01.
Broadening: both use the complex energy z = E + i eta, the same z as the
device matrix, so that the device Green's function is exactly the infinite
system's restricted to the device.
"""
from __future__ import annotations

import numpy as np


def fermi(e, mu: float, kt: float):
    x = (np.asarray(e, dtype=np.float64) - mu) / kt
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def transverse_modes(n_transverse: int, t0: float):
    """Hard-wall transverse sine modes phi[x, m] and energies eps[m]
    (eps_m = 2 t0 (1 - cos(m pi / (N + 1))), m = 1..N)."""
    x = np.arange(1, n_transverse + 1)
    m = np.arange(1, n_transverse + 1)
    phi = np.sqrt(2.0 / (n_transverse + 1)) * np.sin(np.outer(x, m) * np.pi / (n_transverse + 1))
    eps = 2.0 * t0 * (1.0 - np.cos(m * np.pi / (n_transverse + 1)))
    return phi, eps


def chain_surface_sigma(w, t0: float):
    """Self-energy t0^2 g_s of a semi-infinite 1-D chain (on-site 2 t0, hopping
    -t0) seen from a site coupled to its end with -t0, at w = z - eps_m.

    g_s solves g = 1 / (w - 2 t0 - t0^2 g); the product of principal square
    roots sqrt(w - 4 t0) sqrt(w) picks the decaying (retarded) root for
    Im z > 0."""
    w = np.asarray(w, dtype=np.complex128)
    return 0.5 * ((w - 2.0 * t0) - np.sqrt(w - 4.0 * t0) * np.sqrt(w))


def fd_lead_sigma(z: complex, n_transverse: int, t0: float) -> np.ndarray:
    """Dense n_transverse x n_transverse retarded self-energy of a hard-wall
    effective-mass lead attached to a contact layer (same for left and right
    by symmetry)."""
    phi, eps = transverse_modes(n_transverse, t0)
    sig_m = chain_surface_sigma(z - eps, t0)
    return (phi * sig_m) @ phi.T


def sancho_rubio(h00: np.ndarray, h01: np.ndarray, z: complex, tol: float = 1e-14,
                 max_iter: int = 100):
    """Surface Green's functions of a semi-infinite periodic lead by
    renormalisation decimation.

    The lead cells are coupled as H_{c,c+1} = h01.  Returns (g_right, g_left):
    g_right is the surface cell Green's function of the lead extending to +inf
    (surface = its first cell), g_left that of the lead extending to -inf
    (surface = its last cell).  Each iteration doubles the cell distance the
    effective couplings span; the loop stops once they fall below tol."""
    m = h00.shape[0]
    eye = np.eye(m)
    alpha = h01.astype(np.complex128).copy()        # effective coupling to the right
    beta = h01.conj().T.astype(np.complex128).copy()  # effective coupling to the left
    eps_bulk = h00.astype(np.complex128).copy()
    eps_r = eps_bulk.copy()   # surface of the right-extending lead
    eps_l = eps_bulk.copy()   # surface of the left-extending lead
    for _ in range(max_iter):
        g = np.linalg.inv(z * eye - eps_bulk)
        agb = alpha @ g @ beta
        bga = beta @ g @ alpha
        eps_r = eps_r + agb
        eps_l = eps_l + bga
        eps_bulk = eps_bulk + agb + bga
        alpha = alpha @ g @ alpha
        beta = beta @ g @ beta
        if max(np.abs(alpha).max(), np.abs(beta).max()) < tol:
            break
    g_right = np.linalg.inv(z * eye - eps_r)
    g_left = np.linalg.inv(z * eye - eps_l)
    return g_right, g_left


def tube_lead_sigmas(z: complex, h00: np.ndarray, h01: np.ndarray):
    """Retarded self-energies of the left and right pristine leads on the first
    and last device cell.  Left lead cells ..., -2, -1 couple to device cell 0
    through H_{-1,0} = h01; right lead cells N, N+1, ... to device cell N-1
    through H_{N-1,N} = h01."""
    g_right, g_left = sancho_rubio(h00, h01, z)
    sig_l = h01.T @ g_left @ h01
    sig_r = h01 @ g_right @ h01.T
    return sig_l, sig_r


def gamma(sigma: np.ndarray) -> np.ndarray:
    """Broadening Gamma = i (Sigma - Sigma+)."""
    return 1j * (sigma - sigma.conj().T)


def sigma_lesser(sigma: np.ndarray, f: float) -> np.ndarray:
    """Lesser self-energy of a contact in equilibrium: i f Gamma
    (skew-Hermitian; purely imaginary when Sigma is complex symmetric)."""
    return 1j * f * gamma(sigma)


def contact_self_energies(device, energies, eta: float, mu=(0.0, 0.0), kt: float = 0.025):
    """Retarded and lesser self-energies of both contacts at every energy.

    Returns four complex128 arrays [nE, nc, nc]: sigL, sigR, sig_lessL, sig_lessR,
    in the site order of device.contacts[0] / device.contacts[1]."""
    energies = np.asarray(energies, dtype=np.float64)
    ne = energies.size
    ncl, ncr = len(device.contacts[0]), len(device.contacts[1])
    sl = np.zeros((ne, ncl, ncl), np.complex128)
    sr = np.zeros((ne, ncr, ncr), np.complex128)
    for k, e in enumerate(energies):
        z = complex(e, eta)
        if device.lead["kind"] == "fd_modes":
            s = fd_lead_sigma(z, device.lead["n_transverse"], device.lead["t0"])
            sl[k], sr[k] = s, s
        elif device.lead["kind"] == "sancho_rubio":
            sl[k], sr[k] = tube_lead_sigmas(z, device.lead["h00"], device.lead["h01"])
        else:
            raise ValueError(device.lead["kind"])
    fl = fermi(energies, mu[0], kt)
    fr = fermi(energies, mu[1], kt)
    ll = np.stack([sigma_lesser(sl[k], fl[k]) for k in range(ne)]) if ne else sl.copy()
    lr = np.stack([sigma_lesser(sr[k], fr[k]) for k in range(ne)]) if ne else sr.copy()
    return sl, sr, ll, lr
