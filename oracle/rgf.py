"""Plain recursive Green's function method over transport layers.

Section 2 reviews RGF as two passes: fold the layers to the left into the
current one (left to right), then extract diagonal and nearest off-diagonal
blocks (right to left).  Here layers are the blocks q = 0..N-1 of the
block-tridiagonal A, with a_q = A_{q,q+1} and abar_q = A_{q+1,q}.

Retarded (left-connected g_q, then full G):
    g_0 = A_00^{-1},   g_q = (A_qq - abar_{q-1} g_{q-1} a_{q-1})^{-1}
    G_{N-1} = g_{N-1}, G_qq = g_q + g_q a_q G_{q+1} abar_q g_q,
    G_{q,q+1} = -g_q a_q G_{q+1}
Lesser (Sigma^< block diagonal over layers):
    g^<_0 = g_0 S_0 g_0+,  g^<_q = g_q (S_q + abar_{q-1} g^<_{q-1} abar_{q-1}+) g_q+
    G^<_{N-1} = g^<_{N-1},
    G^<_qq = g^<_q + g_q a_q G^<_{q+1} a_q+ g_q+ - (Y - Y+),
    Y = G_{q,q+1} abar_q g^<_q.
The lesser backward step follows from the Keldysh relation
G^< = (I - G W) g^< (I - W+ G+) for the cut between layers q and q+1 (W the
coupling blocks); g^< skew-Hermitian turns the cross terms into -(Y - Y+).
"""
from __future__ import annotations

import numpy as np


def _block(hcsr, rows, cols):
    return hcsr[rows][:, cols].toarray()


def diag_greens(h, v, energies, eta: float, layers, contacts, sig_r, sig_less):
    """diag G^r, G^<, G^> for a device whose H couples only consecutive layers.

    h: scipy sparse (or dense) H; layers: list of site arrays in transport
    order; contacts: site arrays of the contacts, each equal (as a set) to the
    first or last layer; sig_r / sig_less: lists of [nE, nc, nc] arrays.
    Returns three complex128 arrays [nE, n]."""
    import scipy.sparse as sp
    hcsr = sp.csr_matrix(h) if not sp.issparse(h) else h.tocsr()
    n = hcsr.shape[0]
    nl = len(layers)
    v = np.zeros(n) if v is None else np.asarray(v, dtype=np.float64)
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    # energy-independent blocks
    hqq = [_block(hcsr, L, L) for L in layers]
    vq = [v[L] for L in layers]
    aq = [-_block(hcsr, layers[q], layers[q + 1]) for q in range(nl - 1)]      # A_{q,q+1}
    abq = [-_block(hcsr, layers[q + 1], layers[q]) for q in range(nl - 1)]     # A_{q+1,q}
    # contact placement: which layer and the permutation into layer order
    place = []
    for sites in contacts:
        sites = np.asarray(sites)
        hit = None
        for q in (0, nl - 1):
            if set(sites.tolist()) == set(np.asarray(layers[q]).tolist()):
                hit = q
        if hit is None:
            raise ValueError("contact sites must form the first or last layer")
        pos = {s: i for i, s in enumerate(np.asarray(layers[hit]).tolist())}
        perm = np.array([pos[s] for s in sites.tolist()])
        place.append((hit, perm))

    ne = energies.size
    dgr = np.zeros((ne, n), np.complex128)
    dgl = np.zeros((ne, n), np.complex128)
    for k, e in enumerate(energies):
        z = complex(e, eta)
        aqq = []
        sq = [None] * nl
        for q in range(nl):
            m = len(layers[q])
            aqq.append(z * np.eye(m) - hqq[q] - np.diag(vq[q]))
        for c, (q, perm) in enumerate(place):
            m = len(layers[q])
            sig = np.zeros((m, m), np.complex128)
            sig[np.ix_(perm, perm)] = sig_r[c][k]
            aqq[q] = aqq[q] - sig
            sl = np.zeros((m, m), np.complex128)
            sl[np.ix_(perm, perm)] = sig_less[c][k]
            sq[q] = sl if sq[q] is None else sq[q] + sl
        # forward (fold) pass
        g = [None] * nl
        gl = [None] * nl
        for q in range(nl):
            m = aqq[q]
            if q > 0:
                m = m - abq[q - 1] @ g[q - 1] @ aq[q - 1]
            g[q] = np.linalg.inv(m)
            src = np.zeros_like(m) if sq[q] is None else sq[q].copy()
            if q > 0:
                src = src + abq[q - 1] @ gl[q - 1] @ abq[q - 1].conj().T
            gl[q] = g[q] @ src @ g[q].conj().T
        # backward (extract) pass
        G = g[nl - 1]
        GL = gl[nl - 1]
        dgr[k, layers[nl - 1]] = np.diag(G)
        dgl[k, layers[nl - 1]] = np.diag(GL)
        for q in range(nl - 2, -1, -1):
            g_off = -g[q] @ aq[q] @ G                      # G_{q,q+1}
            G_new = g[q] + g[q] @ aq[q] @ G @ abq[q] @ g[q]
            Y = g_off @ abq[q] @ gl[q]
            GL_new = gl[q] + g[q] @ aq[q] @ GL @ aq[q].conj().T @ g[q].conj().T - (Y - Y.conj().T)
            G, GL = G_new, GL_new
            dgr[k, layers[q]] = np.diag(G)
            dgl[k, layers[q]] = np.diag(GL)
    dgg = dgl + dgr - dgr.conj()
    return dgr, dgl, dgg
