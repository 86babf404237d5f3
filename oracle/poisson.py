"""Newton step of the Schroedinger-Poisson problem -- oracle.

TEST INFRASTRUCTURE (see oracle/__init__.py): only tests/, smoke() and
bench.py's cpu_baseline may use it.

The density n(V) of Section 1 depends on the on-site potential V through A;
the potential in turn follows Poisson's equation.  On the device's sites, with
a symmetric positive definite discrete Poisson operator K, a coupling beta
and a background (doping) density n_D:

  F(V) = K V - beta (n(V) - n_D),   J(V) = dF/dV = K - beta chi,
  chi_kj = d n_k / d V_j,

and the Newton step solves J delta = -F.  chi is the density's
vector-Jacobian product with unit cotangents (row k of chi is J^T e_k of the
density map), formed for all rows at once, then J delta = -F is solved
densely: no symmetry of chi is assumed here.
"""
from __future__ import annotations

import numpy as np

from . import definition, gradient


def residual(h, v, energies, eta, contacts, sig_r, sig_less, cweights, K, beta, nd):
    n = gradient.density(h, v, energies, eta, contacts, sig_r, sig_less, cweights)
    return np.asarray(K) @ np.asarray(v) - beta * (n - np.asarray(nd))


def response(h, v, energies, eta, contacts, sig_r, sig_less, cweights):
    """chi[k, j] = d n_k / d V_j: the density's vector-Jacobian product
    (gradient.density_vjp) with the cotangent e_k gives row k,
    chi[k, j] = sum_E c_E Re[-i (G_kj G^<_jk + G^<_kj conj(G_kj))];
    all rows are formed from the same G and G^< of each energy."""
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    m = definition.dense_h(h).shape[0]
    chi = np.zeros((m, m))
    for k, e in enumerate(energies):
        g, gl = definition.full_greens(h, v, e, eta, contacts, [s[k] for s in sig_r],
                                       [s[k] for s in sig_less])
        term = g * gl.T + gl * g.conj()
        chi += cweights[k] * np.real(-1j * term)
    return chi


def newton_step(h, v, energies, eta, contacts, sig_r, sig_less, cweights, K, beta, nd):
    """Returns (delta, F(V)) with J(V) delta = -F(V)."""
    F = residual(h, v, energies, eta, contacts, sig_r, sig_less, cweights, K, beta, nd)
    J = np.asarray(K) - beta * response(h, v, energies, eta, contacts, sig_r, sig_less, cweights)
    return np.linalg.solve(J, -F), F
