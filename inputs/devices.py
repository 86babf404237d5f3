"""Device Hamiltonians: 2-D effective-mass finite-difference grids and a
zigzag carbon-nanotube tight-binding model.

Section 2 describes the device as N_y layers of N_x points, a five-point
stencil giving a symmetric block-tridiagonal H, and two semi-infinite leads
whose effect is folded into the first and last layer.  Section 4.2 uses a
continuum (effective-mass) superlattice and a tight-binding carbon structure.
Everything here is deterministic given its seed.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# hbar^2 / (2 m_0) in eV nm^2
HBAR2_2M0 = 0.0380998


@dataclasses.dataclass
class Device:
    """A device Hamiltonian and its geometry.

    rowptr/col/val: CSR of the real symmetric H (full pattern, diagonal
    included), sites numbered 0..n-1.
    coords: (n, 3) site positions in nm; axis 0 is the transport direction.
    layers: list of site-index arrays in transport order; H couples only
    consecutive layers (the block-tridiagonal structure of Section 2).
    contacts: site arrays of the left and right contact layers (the sites the
    dense lead self-energies act on).
    lead: data needed to build the lead self-energies (model specific).
    """

    name: str
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    coords: np.ndarray
    layers: list
    contacts: list
    lead: dict

    def dense_h(self) -> np.ndarray:
        h = np.zeros((self.n, self.n))
        for i in range(self.n):
            for p in range(self.rowptr[i], self.rowptr[i + 1]):
                h[i, self.col[p]] += self.val[p]
        return h

    def scipy_h(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def _csr_from_triplets(n, rows, cols, vals):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    # merge duplicates
    key = rows * n + cols
    uniq, first = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, first) if len(vals) else vals
    r = (uniq // n).astype(np.int64)
    c = (uniq % n).astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, c, summed.astype(np.float64)


def fd_hopping(a_nm: float, m_eff: float) -> float:
    """t0 = hbar^2 / (2 m* a^2) in eV for grid spacing a (nm)."""
    return HBAR2_2M0 / (m_eff * a_nm * a_nm)


def fd2d(n_transport: int, n_transverse: int, a_nm: float = 0.25, m_eff: float = 0.067,
         potential: np.ndarray | None = None, name: str = "fd2d") -> Device:
    """Five-point effective-mass Hamiltonian on an n_transport x n_transverse
    grid with hard transverse walls (Section 2, Fig. 1-2).

    Site (y, x) -> y * n_transverse + x, y along transport.  On-site 4 t0 + V,
    nearest-neighbour hopping -t0.  The first and last layers are the contact
    layers coupled to semi-infinite leads of the same cross-section (at V=0).
    """
    t0 = fd_hopping(a_nm, m_eff)
    ny, nx = n_transport, n_transverse
    n = ny * nx
    v = np.zeros(n) if potential is None else np.asarray(potential, dtype=np.float64).reshape(n)
    idx = np.arange(n).reshape(ny, nx)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [4.0 * t0 + v]
    # transverse bonds
    a, b = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    rows += [a, b]; cols += [b, a]; vals += [np.full(a.size, -t0)] * 2
    # longitudinal bonds
    a, b = idx[:-1, :].ravel(), idx[1:, :].ravel()
    rows += [a, b]; cols += [b, a]; vals += [np.full(a.size, -t0)] * 2
    rowptr, col, val = _csr_from_triplets(n, np.concatenate(rows), np.concatenate(cols),
                                          np.concatenate(vals))
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    coords = np.stack([yy.ravel() * a_nm, xx.ravel() * a_nm, np.zeros(n)], axis=1)
    layers = [idx[y].copy() for y in range(ny)]
    contacts = [idx[0].astype(np.int32).copy(), idx[ny - 1].astype(np.int32).copy()]
    lead = {"kind": "fd_modes", "t0": t0, "n_transverse": nx, "a_nm": a_nm, "m_eff": m_eff}
    return Device(name, n, rowptr, col, val, coords, layers, contacts, lead)


# ---------------------------------------------------------------------------
# zigzag (n,0) carbon nanotube, nearest-neighbour tight binding
# ---------------------------------------------------------------------------

A_CC_NM = 0.142


def _zigzag_rings(n_rings: int, n: int):
    """Bond list of a zigzag (n,0) tube made of n_rings atomic rings of n atoms.

    Ring k, atom j -> k*n + j.  Rings 2m -> 2m+1 are joined by zigzag bonds
    (every atom to two atoms of the next ring), rings 2m+1 -> 2m+2 by axial
    bonds (one to one).  Angular offsets repeat every four rings, so the
    translational cell holds 4n atoms.
    """
    bonds = []
    # angular offset (in units of 2 pi / n) of each ring: 0, 1/2, 1/2, 0, 0, 1/2, ...
    def offset(k):
        return 0.5 if (k % 4) in (1, 2) else 0.0
    for k in range(n_rings - 1):
        if k % 2 == 0:  # zigzag bonds
            for j in range(n):
                if offset(k) == 0.0:  # atom j at angle j -> next-ring atoms at j-1/2, j+1/2
                    nb = [(j - 1) % n, j]
                else:  # atom j at angle j+1/2 -> next-ring atoms at j, j+1
                    nb = [j, (j + 1) % n]
                for jj in nb:
                    bonds.append((k * n + j, (k + 1) * n + jj))
        else:  # axial bonds
            for j in range(n):
                bonds.append((k * n + j, (k + 1) * n + j))
    z = np.zeros(n_rings)
    for k in range(1, n_rings):
        z[k] = z[k - 1] + (A_CC_NM / 2 if (k - 1) % 2 == 0 else A_CC_NM)
    radius = np.sqrt(3.0) * A_CC_NM * n / (2 * np.pi)
    coords = np.zeros((n_rings * n, 3))
    for k in range(n_rings):
        for j in range(n):
            th = 2 * np.pi * (j + offset(k)) / n
            coords[k * n + j] = (z[k], radius * np.cos(th), radius * np.sin(th))
    return bonds, coords


def zigzag_tube_blocks(n: int = 10, t: float = -2.7):
    """Pristine cell blocks (H00, H01) of the (n,0) tube, cell = 4 rings.

    H01 couples cell c to cell c+1 (rows: cell c, columns: cell c+1)."""
    bonds, _ = _zigzag_rings(8, n)
    m = 4 * n
    h00 = np.zeros((m, m))
    h01 = np.zeros((m, m))
    for a, b in bonds:
        ca, cb = a // m, b // m
        if ca == 0 and cb == 0:
            h00[a, b] = h00[b, a] = t
        elif ca == 0 and cb == 1:
            h01[a, b - m] = t
        elif ca == 1 and cb == 0:
            h01[b, a - m] = t
    return h00, h01


def zigzag_tube(n_cells: int, n: int = 10, t: float = -2.7, disorder: float = 0.2,
                seed: int = 4, name: str = "zigzag_tube") -> Device:
    """(n,0) zigzag nanotube of n_cells translational cells (4 n atoms each)
    with Anderson on-site disorder uniform in [-disorder, disorder] eV.

    The first and last cells are the contact cells; the leads are pristine
    semi-infinite tubes (blocks from zigzag_tube_blocks)."""
    rng = np.random.default_rng(seed)
    n_rings = 4 * n_cells
    bonds, coords = _zigzag_rings(n_rings, n)
    natom = n_rings * n
    eps = rng.uniform(-disorder, disorder, natom) if disorder > 0 else np.zeros(natom)
    rows = [np.arange(natom)]
    cols = [np.arange(natom)]
    vals = [eps]
    b = np.array(bonds, dtype=np.int64)
    rows += [b[:, 0], b[:, 1]]
    cols += [b[:, 1], b[:, 0]]
    vals += [np.full(len(b), t)] * 2
    rowptr, col, val = _csr_from_triplets(natom, np.concatenate(rows), np.concatenate(cols),
                                          np.concatenate(vals))
    m = 4 * n
    layers = [np.arange(c * m, (c + 1) * m) for c in range(n_cells)]
    contacts = [layers[0].astype(np.int32).copy(), layers[-1].astype(np.int32).copy()]
    h00, h01 = zigzag_tube_blocks(n, t)
    lead = {"kind": "sancho_rubio", "h00": h00, "h01": h01}
    return Device(name, natom, rowptr, col, val, coords, layers, contacts, lead)


# ---------------------------------------------------------------------------
# armchair graphene nanoribbon, nearest-neighbour tight binding (the
# honeycomb stencil: each atom and its three neighbours)
# ---------------------------------------------------------------------------

def _armchair_cells(n_cells: int, n_lines: int):
    """Atom positions (nm) of an armchair ribbon of n_lines dimer lines,
    n_cells translational cells of length 3 a_cc along x (transport), and
    its bonds (pairs at distance a_cc).  Dimer line m sits at y = m sqrt(3)/2
    a_cc; even lines hold atoms at x = 0 and a_cc of each cell, odd lines at
    1.5 and 2.5 a_cc.  Cell c, line m, atom q -> c * 2 n_lines + 2 m + q."""
    a = A_CC_NM
    pos = []
    for c in range(n_cells):
        for m in range(n_lines):
            x0 = 3 * a * c + (0.0 if m % 2 == 0 else 1.5 * a)
            for q in range(2):
                pos.append((x0 + q * a, m * np.sqrt(3.0) / 2 * a, 0.0))
    pos = np.array(pos)
    per = 2 * n_lines
    bonds = []
    for i in range(len(pos)):
        c = i // per
        for j in range(i + 1, min(len(pos), (c + 2) * per)):
            if abs(np.linalg.norm(pos[i] - pos[j]) - a) < 1e-6:
                bonds.append((i, j))
    return bonds, pos


def armchair_ribbon_blocks(n_lines: int = 7, t: float = -2.7):
    """Pristine cell blocks (H00, H01) of the armchair ribbon; H01 couples
    cell c (rows) to cell c + 1 (columns)."""
    bonds, _ = _armchair_cells(3, n_lines)
    m = 2 * n_lines
    h00 = np.zeros((m, m))
    h01 = np.zeros((m, m))
    for a_, b_ in bonds:
        ca, cb = a_ // m, b_ // m
        if ca == 1 and cb == 1:
            h00[a_ - m, b_ - m] = h00[b_ - m, a_ - m] = t
        elif ca == 1 and cb == 2:
            h01[a_ - m, b_ - 2 * m] = t
    return h00, h01


def armchair_ribbon(n_cells: int, n_lines: int = 7, t: float = -2.7, disorder: float = 0.0,
                    vacancies: float = 0.0, seed: int = 6, name: str = "armchair_ribbon") -> Device:
    """Armchair graphene nanoribbon of n_lines dimer lines and n_cells cells
    (2 n_lines atoms each), Anderson on-site disorder uniform in
    [-disorder, disorder] eV, and a fraction `vacancies` of the atoms of the
    inner cells removed (seeded): an irregular honeycomb graph.  The first
    and last cells are the contacts; the leads are pristine ribbons."""
    rng = np.random.default_rng(seed)
    bonds, pos = _armchair_cells(n_cells, n_lines)
    per = 2 * n_lines
    keep = np.ones(len(pos), bool)
    if vacancies > 0:
        inner = np.arange(per, len(pos) - per)
        keep[rng.choice(inner, int(round(vacancies * inner.size)), replace=False)] = False
    new = -np.ones(len(pos), np.int64)
    new[keep] = np.arange(int(keep.sum()))
    natom = int(keep.sum())
    b = np.array([(new[i], new[j]) for i, j in bonds if keep[i] and keep[j]], dtype=np.int64)
    eps = rng.uniform(-disorder, disorder, natom) if disorder > 0 else np.zeros(natom)
    rowptr, col, val = _csr_from_triplets(natom, np.concatenate([np.arange(natom), b[:, 0], b[:, 1]]),
                                          np.concatenate([np.arange(natom), b[:, 1], b[:, 0]]),
                                          np.concatenate([eps, np.full(2 * len(b), t)]))
    cell = np.arange(len(pos)) // per
    layers = [new[(cell == c) & keep] for c in range(n_cells)]
    contacts = [layers[0].astype(np.int32).copy(), layers[-1].astype(np.int32).copy()]
    h00, h01 = armchair_ribbon_blocks(n_lines, t)
    lead = {"kind": "sancho_rubio", "h00": h00, "h01": h01}
    return Device(name, natom, rowptr, col, val, pos[keep], layers, contacts, lead)


# ---------------------------------------------------------------------------
# potentials
# ---------------------------------------------------------------------------

def superlattice_potential(n_transport: int, n_transverse: int, flat: int = 20, well: int = 20,
                           barrier: int = 8, height: float = 0.30, noise: float = 0.010,
                           seed: int = 2) -> np.ndarray:
    """Quantum-well superlattice profile along transport (Section 4.2.1):
    flat ends, then repeating [well | barrier] layers, plus i.i.d. uniform
    on-site noise in [-noise, noise] eV on every device site."""
    rng = np.random.default_rng(seed)
    prof = np.zeros(n_transport)
    period = well + barrier
    for y in range(flat, n_transport - flat):
        if (y - flat) % period >= well:
            prof[y] = height
    v = np.repeat(prof, n_transverse).reshape(n_transport, n_transverse)
    if noise > 0:
        v = v + rng.uniform(-noise, noise, v.shape)
    return v.ravel()


def barrier_potential(n_transport: int, n_transverse: int, rng: np.random.Generator) -> np.ndarray:
    """Random barrier profile: 1-8 barriers of 4-16 layers, heights in
    [0.05, 0.4] eV, placed inside [20, n_transport - 20)."""
    prof = np.zeros(n_transport)
    nb = int(rng.integers(1, 9))
    lo, hi = 20, max(21, n_transport - 20)
    for _ in range(nb):
        w = int(rng.integers(4, 17))
        h = float(rng.uniform(0.05, 0.4))
        s = int(rng.integers(lo, max(lo + 1, hi - w)))
        prof[s:min(s + w, hi)] = h
    return np.repeat(prof, n_transverse)


def smooth_random_potential(n_transport: int, n_transverse: int, amplitude: float = 0.050,
                            sigma: float = 8.0, seed: int = 5) -> np.ndarray:
    """Seeded smooth random on-site potential: uniform noise filtered with a
    Gaussian of width sigma sites, scaled to max |V| = amplitude eV; the two
    contact layers are kept at zero so the leads match the device ends."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    v = gaussian_filter(rng.uniform(-1.0, 1.0, (n_transport, n_transverse)), sigma, mode="nearest")
    v *= amplitude / np.max(np.abs(v))
    v[0, :] = 0.0
    v[-1, :] = 0.0
    return v.ravel()
