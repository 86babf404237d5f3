"""Parity at the full sizes of the two remaining workloads, on sampled
energies against the RGF oracle (swept in both directions; the smaller
error counts, as one direction can itself lose digits at a resonance).

- 64 uneven 2-D devices (widths 32..128, lengths 256..2048, barriers), 128
  energies each, leaf size per width class picked by the autotuner, solved
  by one captured graph (ndg_batch_solve);
- the (10,0) tube of 2000 cells (80 000 orbitals), 256 energies.

Both on the open slab chain (tree kind 3: every folded region holds a
contact or is a thin slab): the 2-D devices with slab and leaf per width
class from the autotuner, the tube as the chain of its 40-atom cells.
Tolerance: helpers.bound_vs_rgf -- 1e-10 plus twice the oracle's own
disagreement between its two sweeps; every sampled energy is printed first.
"""
import sys
import time

import numpy as np
import pytest

from inputs import workloads

from .helpers import bound_vs_rgf, rgf_pool_map

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _err(gr, gl, ref):
    (rgr, rgl) = ref
    return max(np.max(np.abs(gr - rgr)) / np.max(np.abs(rgr)),
               np.max(np.abs(gl - rgl)) / np.max(np.abs(rgl)))


def test_batch_of_64_uneven_devices_full_size(lib):
    import torch
    cuda = torch.device("cuda:0")
    nd = 64
    from paper_1305_1070_amd import autotune
    t0 = time.time()
    wls = [workloads.uneven_device(d) for d in range(nd)]
    by_dev = {id(w.device): w for w in wls}

    def sample(dev):
        wl = by_dev[id(dev)]
        idx = np.linspace(0, len(wl.energies) - 1, 8).round().astype(int)
        sl, sr, ll, lr = wl.self_energies(wl.energies[idx])
        return (torch.tensor(wl.energies[idx], device=cuda),
                [torch.from_numpy(a).to(cuda) for a in (sl, sr)],
                [torch.from_numpy(a).to(cuda) for a in (ll, lr)])

    shape = autotune.tune_classes([w.device for w in wls], sample, wls[0].eta, verbose=True,
                                  candidates=(16, 24), slabs=(8, 12))
    _say("  autotuned (slab, leaf) per width: %s (%.1fs)" % (shape, time.time() - t0))
    plans, ins, grow = [], [], []
    for d in range(nd):
        wl = wls[d]
        dev = wl.device
        slab, leaf = shape[len(dev.contacts[0])]
        sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords,
                          leaf_max=leaf, tree_kind=3, slab=slab, layers=dev.layers)
        plans.append(lib.Plan(sym, max_batch=4))  # 32 graph replays cover 128 energies
        sl, sr, ll, lr = wl.self_energies()
        ins.append((torch.tensor(wl.energies, device=cuda), wl.eta,
                    [torch.from_numpy(a).to(cuda) for a in (sl, sr)],
                    [torch.from_numpy(a).to(cuda) for a in (ll, lr)], None))
        grow.append(torch.zeros(len(wl.energies), dtype=torch.float64, device=cuda))
        if d % 16 == 15:
            _say("  set up %d devices (%.1fs)" % (d + 1, time.time() - t0))
    batch = lib.Batch(plans)
    outs = batch.solve(ins, growth=grow)  # capture + first launch
    torch.cuda.synchronize()
    t1 = time.time()
    outs = batch.solve(ins, growth=grow)  # replay
    torch.cuda.synchronize()
    dt = time.time() - t1
    _say("batch of %d devices x 128 energies: %.3f s per graph launch (%.0f device-energies/s)"
         % (nd, dt, nd * 128 / dt))
    for p in plans:
        assert p.status()[0] == 0
    rng = np.random.default_rng(64)
    pick = [int(rng.integers(128)) for _ in range(nd)]
    jobs = [("uneven_device", {"d": d}, pick[d]) for d in range(nd)]
    got = {}
    for d in range(nd):
        k = pick[d]
        got[d] = (outs[d][0][k].cpu().numpy(), outs[d][1][k].cpu().numpy(),
                  float(grow[d][k].item()))
    del outs, batch
    res = rgf_pool_map(jobs)
    bad = []
    errs = []
    for d in range(nd):
        k = pick[d]
        gr, gl, g = got[d]
        e = min(_err(gr, gl, res[d][1]), _err(gr, gl, res[d][2]))
        dr = _err(res[d][1][0], res[d][1][1], res[d][2])
        bound = bound_vs_rgf(dr)
        _say("  device %2d E[%3d] growth %.3e err %.2e rgf fwd/rev %.1e bound %.1e"
             % (d, k, g, e, dr, bound))
        errs.append(e)
        if not e < bound:
            bad.append(d)
    errs = np.array(errs)
    _say("  errors above 1e-10: %d, above 1e-6: %d, median %.1e, worst %.1e"
         % (np.sum(errs > 1e-10), np.sum(errs > 1e-6), np.median(errs), errs.max()))
    assert not bad, bad


def test_tube_2000_cells_full_size(lib):
    import torch
    wl = workloads.nanotube()
    dev = wl.device
    cuda = torch.device("cuda:0")
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, tree_kind=3,
                      slab=-1, layers=dev.layers)
    plan = lib.Plan(sym, max_batch=256)
    sl, sr, ll, lr = wl.self_energies()
    E = torch.tensor(wl.energies, device=cuda)
    sig_r = [torch.from_numpy(a).to(cuda) for a in (sl, sr)]
    sig_l = [torch.from_numpy(a).to(cuda) for a in (ll, lr)]
    growth = torch.zeros(len(wl.energies), dtype=torch.float64, device=cuda)
    plan.solve(E, wl.eta, sig_r, sig_l, growth=growth)
    torch.cuda.synchronize()
    t1 = time.time()
    gr, gl, gg = plan.solve(E, wl.eta, sig_r, sig_l, growth=growth)
    torch.cuda.synchronize()
    dt = time.time() - t1
    _say("tube 2000 cells, 256 energies: %.3f s (%.0f energies/s)" % (dt, 256 / dt))
    assert plan.status()[0] == 0
    idx = [int(i) for i in np.linspace(3, 252, 8).round()]
    jobs = [("nanotube", {}, i) for i in idx]
    res = dict(zip(idx, rgf_pool_map(jobs)))
    g = growth.cpu().numpy()
    bad = []
    for i in idx:
        a, b = gr[i].cpu().numpy(), gl[i].cpu().numpy()
        e = min(_err(a, b, res[i][1]), _err(a, b, res[i][2]))
        dr = _err(res[i][1][0], res[i][1][1], res[i][2])
        bound = bound_vs_rgf(dr)
        _say("  E[%3d]=%.4f growth %.3e err %.2e rgf fwd/rev %.1e bound %.1e"
             % (i, wl.energies[i], g[i], e, dr, bound))
        if not e < bound:
            bad.append(i)
    assert not bad, bad
