"""Gradient of the electron density with respect to the on-site potential,
from the dense definition.

Density n_i = sum_E c_E (-i G^<_ii(E)).  With A = zI - H - diag(V) - Sigma,
dA/dV_k = -e_k e_k^T, so dG^r = G^r e_k e_k^T G^r and
dG^< = dG^r Sigma^< G^r+ + G^r Sigma^< dG^r+ = G^r e_k e_k^T G^< + G^< e_k e_k^T G^r+.
For a cotangent nbar on n, the vector-Jacobian product is
    Vbar_k = sum_E c_E sum_i nbar_i (-i) (G_ik G^<_ki + G^<_ik conj(G_ik))
           = sum_E c_E 2 Im[ (G^< Lambda G^r)_kk ],   Lambda = diag(nbar),
using G^r = (G^r)^T (A complex symmetric) and (G^<)+ = -G^<.  The code
evaluates the first (unsimplified) form.
"""
from __future__ import annotations

import numpy as np

from . import definition


def density_vjp(h, v, energies, eta, contacts, sig_r, sig_less, cweights, nbar):
    """Vbar = J^T nbar for n(V) at the given energies (dense; small devices)."""
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    nbar = np.asarray(nbar, dtype=np.float64)
    out = np.zeros(nbar.size)
    for k, e in enumerate(energies):
        g, gl = definition.full_greens(h, v, e, eta, contacts, [s[k] for s in sig_r],
                                       [s[k] for s in sig_less])
        # term_ik = G_ik G^<_ki + G^<_ik conj(G_ik); Vbar_k += c_E sum_i nbar_i (-i) term_ik
        term = g * gl.T + gl * g.conj()
        out += cweights[k] * np.real(-1j * (nbar[:, None] * term).sum(axis=0))
    return out


def density(h, v, energies, eta, contacts, sig_r, sig_less, cweights):
    _, dgl, _ = definition.diag_greens(h, v, energies, eta, contacts, sig_r, sig_less)
    return definition.density(dgl, cweights)
