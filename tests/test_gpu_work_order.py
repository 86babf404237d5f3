"""Workgroup order of the per-cluster kernels.

The per-cluster kernels remap their (items, energies) grid so that each XCD
takes every eighth energy, in groups of eight energies item by item when the
batch holds a multiple of 64 energies, one energy at a time when it holds a
multiple of 8, and keep the plain order otherwise.  The remap has to be a
bijection of the grid: the same energies solved in batches of 64, 16 and 12
(one batch size per order) must agree bit for bit, and agree with the RGF
oracle.
"""
import sys

import numpy as np
import pytest

from inputs import workloads

from .helpers import gpu_solve, layer_tree, oracle_rgf, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_three_workgroup_orders_agree_bit_for_bit(lib):
    # 160 x 32 superlattice (slab chain, slabs of 12 layers: their levels lie
    # above the 0-0.5 eV window), 64 energies
    wl = workloads.superlattice(n_transport=160, n_transverse=32, n_energies=64, eta=1e-4)
    outs = {}
    for mb in (64, 16, 12):
        _say("superlattice 160x32, 64 energies, batches of %d" % mb)
        out, status = gpu_solve(lib, wl, max_batch=mb, leaf_max=20, **layer_tree(wl.device, slab=12))
        assert status[0] == 0
        outs[mb] = out
    for mb in (16, 12):
        for name, a, b in zip(("Gr", "Gless", "Ggreater"), outs[64][:3], outs[mb][:3]):
            assert np.array_equal(a, b), "%s differs between batches of 64 and %d" % (name, mb)
    idx = [0, 21, 42, 63]
    ref = oracle_rgf(wl, energies=wl.energies[idx])
    for name, x, r in zip(("Gr", "Gless"), outs[64][:2], ref[:2]):
        err = rel_err(x[idx], r)
        _say("  %s vs RGF: max rel err %.2e" % (name, err.max()))
        assert err.max() < 1e-9
