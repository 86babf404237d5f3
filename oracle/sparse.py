"""The definition at sampled sites, for devices too large for dense inversion.

Same statement as definition.py (Section 1): A = zI - H - diag(V) - Sigma_L
- Sigma_R, G^r = A^{-1}, G^< = G^r Sigma^< G^r+.  A is factored once per
energy by sparse LU with partial pivoting (SuperLU through scipy); row j of
G^r is the solution of A^T x = e_j, which gives G^r_jj = x_j and
G^<_jj = sum_ab x_a Sigma^<_ab conj(x_b) over each contact's sites.  Used for
full-size parity at sampled sites (one solve per sampled site).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def assemble_a(h, v, z: complex, contacts, sig_r):
    """Sparse A = zI - H - diag(V) - sum_c Sigma_c on contact c's sites (CSC)."""
    hcsr = sp.csr_matrix(h) if not sp.issparse(h) else h.tocsr()
    n = hcsr.shape[0]
    diag = np.full(n, z, dtype=np.complex128)
    if v is not None:
        diag -= np.asarray(v, dtype=np.float64)
    a = sp.diags(diag, format="csr") - hcsr.astype(np.complex128)
    rows, cols, vals = [], [], []
    for sites, s in zip(contacts, sig_r):
        sites = np.asarray(sites)
        rr, cc = np.meshgrid(sites, sites, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(-np.asarray(s).ravel())
    if rows:
        a = a + sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                              shape=(n, n))
    return a.tocsc()


def sampled_diag(h, v, energies, eta: float, contacts, sig_r, sig_less, sites):
    """diag G^r and diag G^< at the given sites for every energy.

    sig_r[c], sig_less[c]: [nE, nc, nc].  Returns two complex128 arrays
    [nE, len(sites)]."""
    sites = np.asarray(sites, dtype=np.int64)
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    ne, m = energies.size, sites.size
    gr = np.zeros((ne, m), np.complex128)
    gl = np.zeros((ne, m), np.complex128)
    for k, e in enumerate(energies):
        a = assemble_a(h, v, complex(e, eta), contacts, [s[k] for s in sig_r])
        n = a.shape[0]
        lu = spla.splu(a)
        rhs = np.zeros((n, m), np.complex128)
        rhs[sites, np.arange(m)] = 1.0
        x = lu.solve(rhs, trans="T")       # column q = row sites[q] of G^r
        gr[k] = x[sites, np.arange(m)]
        for cs, s in zip(contacts, sig_less):
            xc = x[np.asarray(cs)]          # [nc, m]: G^r_{j, a}
            gl[k] += np.einsum("aq,ab,bq->q", xc, s[k], xc.conj())
    return gr, gl
