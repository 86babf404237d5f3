"""The problem statement written out densely (Section 1).

A(E) = E I - H - Sigma^r_L - Sigma^r_R - Sigma^r_Phonon (equation defineA),
with E replaced by z = E + i eta and the on-site potential V added to H.
The phonon self-energy is optional and diagonal (one complex value per site
and energy, the case Section 1 assumes), and its lesser part adds to the
contacts' Sigma^<.  G^r solves A G^r = I and G^< solves
A G^< = Sigma^< (G^r)+ (equation defineGless1), so G^< = G^r Sigma^< G^r+.
G^> on the diagonal is taken from G^> - G^< = G^r - G^r+.

Everything is a plain dense computation: assemble A, LU-factor it with
partial pivoting (scipy/LAPACK), solve for the needed columns.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def dense_h(h) -> np.ndarray:
    """H as a dense float64 array (accepts dense arrays, scipy sparse, or an
    object with a dense_h() method)."""
    if hasattr(h, "dense_h"):
        return h.dense_h()
    if hasattr(h, "toarray"):
        return h.toarray().astype(np.float64)
    return np.asarray(h, dtype=np.float64)


def assemble_a(h: np.ndarray, v, z: complex, contacts, sig_r, sig_r_ph=None) -> np.ndarray:
    """A = z I - H - diag(V) - sum_c Sigma^r_c placed on contact c's sites
    - diag(Sigma^r_Phonon) (sig_r_ph: [n] complex, or None)."""
    n = h.shape[0]
    a = -h.astype(np.complex128)
    a[np.diag_indices(n)] += z
    if v is not None:
        a[np.diag_indices(n)] -= np.asarray(v, dtype=np.float64)
    for sites, s in zip(contacts, sig_r):
        a[np.ix_(sites, sites)] -= s
    if sig_r_ph is not None:
        a[np.diag_indices(n)] -= np.asarray(sig_r_ph, dtype=np.complex128)
    return a


def full_greens(h, v, e: float, eta: float, contacts, sig_r, sig_less, sig_r_ph=None,
                sig_less_ph=None):
    """Full matrices (G^r, G^<) at one energy; sig_r / sig_less are lists of
    dense contact blocks in the site order of `contacts`; sig_r_ph /
    sig_less_ph the phonon self-energies' diagonals ([n] each) or None."""
    hd = dense_h(h)
    a = assemble_a(hd, v, complex(e, eta), contacts, sig_r, sig_r_ph)
    lu = sla.lu_factor(a)
    g = sla.lu_solve(lu, np.eye(a.shape[0], dtype=np.complex128))
    n = a.shape[0]
    sl = np.zeros((n, n), np.complex128)
    for sites, s in zip(contacts, sig_less):
        sl[np.ix_(sites, sites)] += s
    if sig_less_ph is not None:
        sl[np.diag_indices(n)] += np.asarray(sig_less_ph, dtype=np.complex128)
    gl = g @ sl @ g.conj().T
    return g, gl


def diag_greens(h, v, energies, eta: float, contacts, sig_r, sig_less, sig_r_ph=None,
                sig_less_ph=None):
    """diag G^r, diag G^<, diag G^> for every energy.

    sig_r[c] and sig_less[c] are [nE, nc, nc] arrays for contact c;
    sig_r_ph / sig_less_ph are [nE, n] diagonals of the phonon self-energies
    (site order of H) or None.  Returns three complex128 arrays [nE, n]."""
    hd = dense_h(h)
    n = hd.shape[0]
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    ne = energies.size
    dgr = np.zeros((ne, n), np.complex128)
    dgl = np.zeros((ne, n), np.complex128)
    eye = np.eye(n, dtype=np.complex128)
    for k, e in enumerate(energies):
        a = assemble_a(hd, v, complex(e, eta), contacts, [s[k] for s in sig_r],
                       None if sig_r_ph is None else sig_r_ph[k])
        lu = sla.lu_factor(a)
        g = sla.lu_solve(lu, eye)
        dgr[k] = np.diag(g)
        acc = np.zeros(n, np.complex128)
        for sites, s in zip(contacts, sig_less):
            gc = g[:, sites]                       # columns of G^r on the contact
            # (G Sigma^< G+)_jj = sum_ab G_ja S_ab conj(G_jb)
            acc += np.einsum("ja,ab,jb->j", gc, s[k], gc.conj())
        if sig_less_ph is not None:
            # diagonal Sigma^<: (G diag(sigma) G+)_jj = sum_m |G_jm|^2 sigma_m
            acc += (np.abs(g) ** 2) @ np.asarray(sig_less_ph[k], dtype=np.complex128)
        dgl[k] = acc
    dgg = dgl + dgr - dgr.conj()
    return dgr, dgl, dgg


def diag_greater(h, v, energies, eta: float, contacts, sig_r, sig_less) -> np.ndarray:
    """diag G^> formed in its own step (Section 2): G^> = G^r Sigma^> G^r+
    with Sigma^> = Sigma^< + Sigma^r - Sigma^r+ on each contact (the lesser
    and greater self-energies differ by the retarded minus the advanced one).
    With broadening eta > 0 in the device this differs from the identity
    G^< + G^r - G^r+ by 2 i eta diag(G^r G^r+).  Returns complex128 [nE, n]."""
    hd = dense_h(h)
    n = hd.shape[0]
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    out = np.zeros((energies.size, n), np.complex128)
    eye = np.eye(n, dtype=np.complex128)
    for k, e in enumerate(energies):
        a = assemble_a(hd, v, complex(e, eta), contacts, [s[k] for s in sig_r])
        g = sla.lu_solve(sla.lu_factor(a), eye)
        for sites, sr, sl in zip(contacts, sig_r, sig_less):
            sg = sl[k] + sr[k] - sr[k].conj().T
            gc = g[:, sites]
            out[k] += np.einsum("ja,ab,jb->j", gc, sg, gc.conj())
    return out


def transmission(h, v, energies, eta: float, contacts, sig_r) -> np.ndarray:
    """Transmission between the first two contacts, T(E) = Tr[Gamma_L G_LR
    Gamma_R G_LR+] with Gamma = i (Sigma^r - Sigma^r+) and G_LR the block of
    G^r between the contacts' sites.  Returns a real array [nE]."""
    hd = dense_h(h)
    n = hd.shape[0]
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    out = np.zeros(energies.size)
    L, R = contacts[0], contacts[1]
    for k, e in enumerate(energies):
        a = assemble_a(hd, v, complex(e, eta), contacts, [s[k] for s in sig_r])
        rhs = np.zeros((n, len(R)), np.complex128)
        rhs[R, np.arange(len(R))] = 1.0
        glr = sla.lu_solve(sla.lu_factor(a), rhs)[L]        # G^r[L, R]
        gl_ = 1j * (sig_r[0][k] - sig_r[0][k].conj().T)
        gr_ = 1j * (sig_r[1][k] - sig_r[1][k].conj().T)
        out[k] = np.trace(gl_ @ glr @ gr_ @ glr.conj().T).real
    return out


def density(dgl: np.ndarray, cweights: np.ndarray) -> np.ndarray:
    """n_i = sum_E c_E (-i G^<_ii(E)) (real part kept; the imaginary part is
    zero up to rounding because G^< is skew-Hermitian)."""
    return np.real(-1j * (np.asarray(cweights)[:, None] * dgl).sum(axis=0))


def terminal_currents(h, v, energies, eta: float, contacts, sig_r, sig_less, sig_r_ph=None,
                      sig_less_ph=None):
    """Current spectral density into the device from each contact, per energy:

      i_c(E) = Tr[Sigma^<_c G^>_cc - Sigma^>_c G^<_cc]

    over contact c's block, with Sigma^> = Sigma^< + Sigma^r - Sigma^r+ and
    G^> = G^< + G^r - G^r+ (in-scattering times empty states minus
    out-scattering times filled states; the terminal current is
    (e/h) times its energy integral).  Returns a real array [nE, ncontacts]."""
    hd = dense_h(h)
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    out = np.zeros((energies.size, len(contacts)))
    for k, e in enumerate(energies):
        g, gl = full_greens(hd, v, e, eta, contacts, [s[k] for s in sig_r], [s[k] for s in sig_less],
                            None if sig_r_ph is None else sig_r_ph[k],
                            None if sig_less_ph is None else sig_less_ph[k])
        gg = gl + g - g.conj().T
        for c, sites in enumerate(contacts):
            ix = np.ix_(sites, sites)
            sl = sig_less[c][k]
            sg = sl + sig_r[c][k] - sig_r[c][k].conj().T
            val = np.trace(sl @ gg[ix] - sg @ gl[ix])
            out[k, c] = val.real
    return out
