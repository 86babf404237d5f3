"""The definition in 50-digit arithmetic (mpmath), without LAPACK.

Same statement as definition.py -- A = zI - H - diag(V) - Sigma_L - Sigma_R
- diag(Sigma_Phonon), G^r = A^{-1}, G^< = G^r Sigma^< G^r+ (Section 1) --
evaluated with mpmath's own Gaussian elimination, for tiny devices (n up to
~30).
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


def diag_greens(h, v, e: float, eta: float, contacts, sig_r, sig_less, dps: int = 50,
                sig_r_ph=None, sig_less_ph=None):
    """diag G^r and diag G^< at one energy, returned as complex128 arrays.

    h: dense float array; sig_r / sig_less: lists of dense contact blocks;
    sig_r_ph / sig_less_ph: per-site phonon self-energies ([n]) or None."""
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    with mp.workdps(dps):
        z = mp.mpc(e, eta)
        a = mp.matrix(n, n)
        for i in range(n):
            for j in range(n):
                a[i, j] = -mp.mpf(h[i, j])
            a[i, i] += z
            if v is not None:
                a[i, i] -= mp.mpf(float(v[i]))
        for sites, s in zip(contacts, sig_r):
            for p, i in enumerate(sites):
                for q, j in enumerate(sites):
                    a[int(i), int(j)] -= mp.mpc(s[p, q].real, s[p, q].imag)
        if sig_r_ph is not None:
            for i in range(n):
                w = complex(sig_r_ph[i])
                a[i, i] -= mp.mpc(w.real, w.imag)
        g = mp.inverse(a)
        dgr = np.array([complex(g[i, i]) for i in range(n)])
        dgl = np.zeros(n, np.complex128)
        for sites, s in zip(contacts, sig_less):
            sm = [[mp.mpc(s[p, q].real, s[p, q].imag) for q in range(len(sites))]
                  for p in range(len(sites))]
            for i in range(n):
                acc = mp.mpc(0)
                for p, a_ in enumerate(sites):
                    gia = g[i, int(a_)]
                    for q, b_ in enumerate(sites):
                        acc += gia * sm[p][q] * mp.conj(g[i, int(b_)])
                dgl[i] += complex(acc)
        if sig_less_ph is not None:
            # a source on site m alone contributes G_im sigma_m conj(G_im)
            for i in range(n):
                acc = mp.mpc(0)
                for m in range(n):
                    w = complex(sig_less_ph[m])
                    acc += g[i, m] * mp.mpc(w.real, w.imag) * mp.conj(g[i, m])
                dgl[i] += complex(acc)
    return dgr, dgl
