"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerance: 1e-10 normwise relative per energy for the FP64 path (the
target stated for the method), on diag G^r, diag G^< and diag G^>.
"""
import sys

import numpy as np
import pytest

from inputs import devices, workloads

from .helpers import gpu_solve, oracle_dense, oracle_rgf, rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check(out, ref, tol=TOL, what=""):
    for name, x, r in zip(("Gr", "Gless", "Ggreater"), out, ref):
        err = rel_err(x, r)
        assert np.all(err < tol), "%s %s: max rel err %.3e" % (what, name, err.max())


@pytest.mark.parametrize("tree_kind", [0, 1, 2])
def test_small_grid_all_tree_kinds(lib, tree_kind):
    wl = workloads.small_grid(12, 8, n_energies=4, emin=0.02, emax=0.4, eta=1e-3, noise=0.05,
                              seed=3)
    _say("small grid 12x8 tree_kind=%d" % tree_kind)
    out, status = gpu_solve(lib, wl, tree_kind=tree_kind, leaf_max=8)
    assert status[0] == 0
    _check(out, oracle_dense(wl), what="tree%d" % tree_kind)


def test_ragged_tiles_and_batching(lib):
    """Odd sizes (clusters and boundaries not multiples of 16/64), more
    energies than the batch, an on-site potential passed separately."""
    wl = workloads.small_grid(37, 21, n_energies=7, emin=0.01, emax=0.5, eta=1e-4, seed=1)
    v = np.random.default_rng(21).uniform(-0.05, 0.05, wl.device.n)
    _say("ragged 37x21, 7 energies, batch 3")
    out, status = gpu_solve(lib, wl, max_batch=3, leaf_max=24, V=v)
    assert status[0] == 0
    _check(out, oracle_dense(wl, V=v), what="ragged")


def test_waveguide_64x32_all_energies(lib):
    wl = workloads.uniform_waveguide()
    _say("waveguide 64x32, 16 energies")
    out, status = gpu_solve(lib, wl)
    assert status[0] == 0
    _check(out, oracle_dense(wl), what="waveguide")


def test_stored_blocks_match_dense(lib):
    """Every stored entry of the G^r and G^< fronts equals the dense
    definition (Section 3.2: G^(0) and P^(0) are incomplete but exact)."""
    from oracle import definition
    wl = workloads.small_grid(10, 6, n_energies=2, emin=0.05, emax=0.3, eta=1e-3, noise=0.02,
                              seed=4)
    dev = wl.device
    _say("stored blocks 10x6")
    out, status, plan, sym = gpu_solve(lib, wl, leaf_max=6, keep_plan=True)
    arr = sym.arrays()
    perm, cl_off, bptr, bidx = arr["perm"], arr["cl_off"], arr["bptr"], arr["bidx"]
    sl, sr, ll, lr = wl.self_energies()
    for k in range(2):
        g, gl = definition.full_greens(dev.scipy_h(), None, wl.energies[k], wl.eta, dev.contacts,
                                       [sl[k], sr[k]], [ll[k], lr[k]])
        for c in range(len(cl_off) - 1):
            pts = np.concatenate([np.arange(cl_off[c], cl_off[c + 1]), bidx[bptr[c]:bptr[c + 1]]])
            orig = perm[pts]
            f = len(pts)
            s = cl_off[c + 1] - cl_off[c]
            fg = plan.export_block(2, k, c, (f, f))
            fp = plan.export_block(3, k, c, (f, f))
            ref_g = g[np.ix_(orig, orig)]
            ref_p = gl[np.ix_(orig, orig)]
            # rows of the cluster (its own rows and its boundary columns) are final
            scale_g = np.max(np.abs(ref_g[:s]))
            scale_p = max(np.max(np.abs(ref_p[:s])), 1e-300)
            assert np.max(np.abs(fg[:s] - ref_g[:s])) < TOL * scale_g
            assert np.max(np.abs(fp[:s] - ref_p[:s])) < TOL * max(scale_p, np.max(np.abs(gl)))


def test_superlattice_full_size_sampled_energies(lib):
    """1024 x 64 superlattice at its full size; four of the 512 energies
    compared with the RGF oracle."""
    wl = workloads.superlattice(n_energies=512)
    idx = [0, 137, 300, 511]
    e = wl.energies[idx]
    _say("superlattice 1024x64 sampled energies %s" % idx)
    out, status = gpu_solve(lib, wl, energies=e, leaf_max=16)
    assert status[0] == 0
    _check(out, oracle_rgf(wl, energies=e), what="superlattice")


def test_tube_vs_rgf(lib):
    wl = workloads.nanotube(n_cells=120, n_energies=5)
    _say("tube 120 cells")
    out, status = gpu_solve(lib, wl, leaf_max=24)
    assert status[0] == 0
    _check(out, oracle_rgf(wl), what="tube")


def test_lesser_invariants_on_gpu_output(lib):
    wl = workloads.small_grid(16, 10, n_energies=3, emin=0.05, emax=0.3, eta=1e-6, seed=8)
    out, status = gpu_solve(lib, wl, leaf_max=10)
    gr, gl, gg = out
    assert np.max(np.abs(gl.real)) < 1e-12 * np.max(np.abs(gl))
    assert np.min((-1j * gl).real) > -1e-12 * np.max(np.abs(gl))
    assert np.allclose(gg - gl, gr - gr.conj(), atol=0, rtol=0)


def test_zero_energies_is_a_noop(lib):
    import torch
    wl = workloads.small_grid(6, 4, n_energies=1)
    dev = wl.device
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords)
    plan = lib.Plan(sym, max_batch=2)
    cuda = torch.device("cuda:0")
    e = torch.zeros(0, dtype=torch.float64, device=cuda)
    s = [torch.zeros((0, 4, 4), dtype=torch.complex128, device=cuda) for _ in range(2)]
    gr, gl, gg = plan.solve(e, 1e-3, s, s)
    torch.cuda.synchronize()
    assert gr.shape == (0, dev.n)
