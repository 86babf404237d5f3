"""Parity on an unstructured stencil: the armchair graphene nanoribbon (the
honeycomb stencil of Section 4.2's carbon devices) with Anderson disorder and
seeded vacancies, an irregular graph.  The separator tree is cut either
geometrically or, without coordinates, by breadth-first level sets (Section
3.2 accepts any partition that obeys its two rules).  Compared with the
dense definition through the C ABI at the FP64 tolerance, 1e-10.
"""
import sys

import numpy as np
import pytest

from inputs import phonons, workloads

from .helpers import TOL, gpu_solve, layer_tree, oracle_dense, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check(out, ref, what):
    gr, gl, gg, growth = out
    er = rel_err(gr, ref[0])
    el = rel_err(gl, ref[1])
    scale = np.maximum(np.max(np.abs(ref[0]), axis=-1), np.max(np.abs(ref[1]), axis=-1))
    eg = np.max(np.abs(gg - ref[2]), axis=-1) / scale
    for k in range(len(growth)):
        _say("  %s energy %d growth %.3e errs %.2e %.2e %.2e" % (what, k, growth[k], er[k], el[k], eg[k]))
    assert np.all(np.maximum(np.maximum(er, el), eg) < TOL)


@pytest.mark.parametrize("tree", ["level_set", "cell_chain"])
def test_armchair_ribbon_matches_definition(lib, tree):
    """The level-set tree (graph only, no coordinates) and the chain of the
    ribbon's cells (its transport layers, rooted in the middle cell)."""
    wl = workloads.armchair_ribbon(n_cells=40, n_energies=6)
    dev = wl.device
    if tree == "level_set":
        sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, None, leaf_max=16)
    else:
        sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords,
                          **layer_tree(dev, slab=-1))
    info = sym.info()
    _say("armchair ribbon n=%d tree=%s clusters %d levels %d" % (dev.n, tree, info["nclusters"],
                                                                  info["max_height"]))
    out, status = gpu_solve(lib, wl, sym=sym)
    assert status[0] == 0
    _check(out, oracle_dense(wl), "agnr %s" % tree)


def test_armchair_ribbon_scattering_graph_tree(lib):
    """Phonon self-energies on every atom with the level-set tree: the
    all-ancestor frames follow whatever tree the graph gives."""
    import torch
    from oracle import definition
    wl = workloads.armchair_ribbon(n_cells=30, n_energies=4)
    dev = wl.device
    e = wl.energies
    sl_, sr_, ll_, lr_ = wl.self_energies(e)
    pr, pl = phonons.diagonal_self_energies(dev, e, gamma0=2e-2, mu=wl.mu, seed=12)
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, None, leaf_max=16)
    plan = lib.Plan(sym, max_batch=4)
    plan.enable_scattering()
    cuda = torch.device("cuda:0")
    E = torch.tensor(e, device=cuda)
    sr = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (sl_, sr_)]
    sl = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (ll_, lr_)]
    growth = torch.zeros(len(e), dtype=torch.float64, device=cuda)
    _say("armchair ribbon scattering, level-set tree, n=%d" % dev.n)
    gr, gl, gg = plan.solve_scattering(E, wl.eta, sr, sl, torch.from_numpy(pr).to(cuda),
                                       torch.from_numpy(pl).to(cuda), growth=growth)
    torch.cuda.synchronize()
    assert plan.status()[0] == 0
    ref = definition.diag_greens(dev.scipy_h(), None, e, wl.eta, dev.contacts, [sl_, sr_], [ll_, lr_],
                                 pr, pl)
    _check((gr.cpu().numpy(), gl.cpu().numpy(), gg.cpu().numpy(), growth.cpu().numpy()), ref,
           "agnr scattering")
