"""Self-consistent Born loop for local elastic phonon scattering -- oracle.

TEST INFRASTRUCTURE (see oracle/__init__.py): only tests/, smoke() and
bench.py's cpu_baseline may use it.

Equation defineA carries a phonon self-energy that Section 1 takes diagonal
and that, in a scattering calculation, depends on the Green's functions
themselves.  The paper fixes no phonon model; this loop takes the local
elastic (deformation-potential, high-temperature) one:

  Sigma^r_ph,k(E) = D0 G^r_kk(E),   Sigma^<_ph,k(E) = D0 G^<_kk(E),

per site k and energy E, iterated from a given start (zero by default):

  1. diag G^r, diag G^< from the definition with the current Sigma_ph;
  2. the new self-energies S' = D0 diag G;
  3. residual = max |S' - S| / max |S'| over both self-energies, all sites
     and energies;
  4. S <- (1 - mix) S + mix S'; stop after this update when residual < tol
     or after max_iter solves.

The Green's functions returned are those of the last solve (with the
self-energies before the last update).
"""
from __future__ import annotations

import numpy as np

from . import definition


def scba(h, v, energies, eta: float, contacts, sig_r, sig_less, d0: float, mix: float, tol: float,
         max_iter: int, sig_r_ph=None, sig_less_ph=None):
    """Returns (dgr, dgl, dgg, sig_r_ph, sig_less_ph, iterations, residual);
    self-energies [nE, n] complex128 in the site order of H."""
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    n = definition.dense_h(h).shape[0]
    shape = (energies.size, n)
    sr = np.zeros(shape, np.complex128) if sig_r_ph is None else np.array(sig_r_ph, np.complex128)
    sl = np.zeros(shape, np.complex128) if sig_less_ph is None else np.array(sig_less_ph, np.complex128)
    it, res = 0, np.inf
    dgr = dgl = dgg = None
    while it < max_iter:
        dgr, dgl, dgg = definition.diag_greens(h, v, energies, eta, contacts, sig_r, sig_less, sr, sl)
        it += 1
        nr, nl = d0 * dgr, d0 * dgl
        scale = max(np.max(np.abs(nr)), np.max(np.abs(nl)))
        diff = max(np.max(np.abs(nr - sr)), np.max(np.abs(nl - sl)))
        res = diff / scale if scale > 0 else 0.0
        sr = (1.0 - mix) * sr + mix * nr
        sl = (1.0 - mix) * sl + mix * nl
        if res < tol:
            break
    return dgr, dgl, dgg, sr, sl, it, res
