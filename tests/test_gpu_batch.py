"""Wide contacts and batched uneven devices, through the C ABI.

Contacts wider than one cluster (96 and 128 sites) span a parent-child chain
of clusters; a batch of devices of uneven widths and lengths is solved by
one graph launch (ndg_batch_solve) and must reproduce, bit for bit, the
per-plan solves, on every replay, and match the oracle.
"""
import sys

import numpy as np
import pytest

from inputs import workloads

from .helpers import TOL, gpu_solve, layer_tree, oracle_dense, oracle_rgf, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _errs(out, ref):
    er = rel_err(out[0], ref[0])
    el = rel_err(out[1], ref[1])
    scale = np.maximum(np.max(np.abs(ref[0]), axis=-1), np.max(np.abs(ref[1]), axis=-1))
    eg = np.max(np.abs(np.atleast_2d(out[2] - ref[2])), axis=-1) / scale
    return np.max(np.stack([er, el, eg]), axis=0)


@pytest.mark.parametrize("length,width", [(40, 96), (24, 128)])
def test_wide_contact_spans_a_chain(lib, length, width):
    """Nested dissection with 64-point clusters: a contact wider than a
    cluster spans a parent-child chain (its self-energy entries go to the
    lower owner's front)."""
    wl = workloads.small_grid(length, width, n_energies=4, emin=0.02, emax=0.45, eta=1e-4,
                              noise=0.03, seed=width)
    _say("wide contact %dx%d" % (length, width))
    out, status, plan, sym = gpu_solve(lib, wl, leaf_max=16, keep_plan=True)
    assert status[0] == 0
    assert sym.info()["max_cluster"] <= 64
    err = _errs(out, oracle_dense(wl))
    for k in range(len(err)):
        _say("  energy %d growth %.3e err %.2e" % (k, out[3][k], err[k]))
    assert np.all(err < TOL)


def _batch_inputs(wls, cuda):
    import torch
    ins, refs = [], []
    for wl in wls:
        sl, sr, ll, lr = wl.self_energies()
        E = torch.tensor(wl.energies, dtype=torch.float64, device=cuda)
        sig_r = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (sl, sr)]
        sig_l = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (ll, lr)]
        V = torch.zeros(wl.device.n, dtype=torch.float64, device=cuda)
        ins.append((E, wl.eta, sig_r, sig_l, V))
    return ins


def _eager(plans, ins):
    import torch
    res = []
    for p, (E, eta, sr, sl, V) in zip(plans, ins):
        gr, gl, gg = p.solve(E, eta, sr, sl, V=V)
        res.append((gr, gl, gg))
    torch.cuda.synchronize()
    return [tuple(t.cpu().numpy() for t in r) for r in res]


def test_batch_of_uneven_devices_replays_match_eager_and_oracle(lib):
    import torch
    cuda = torch.device("cuda:0")
    wls = workloads.uneven_devices(n_devices=5, n_energies=6, lmin=20, lmax=72, eta=1e-4)
    _say("batch of %d devices: %s" % (len(wls), ", ".join(w.name for w in wls)))
    plans = []
    for wl in wls:
        d = wl.device
        sym = lib.analyze(d.n, d.rowptr, d.col, d.val, d.contacts, d.coords, leaf_max=16,
                          **layer_tree(d, 6))
        plans.append(lib.Plan(sym, max_batch=4))  # 6 energies: two batches per device
    ins = _batch_inputs(wls, cuda)
    eager = _eager(plans, ins)
    for wl, out in zip(wls, eager):
        err = _errs(out, oracle_rgf(wl))
        _say("  %s max err vs RGF %.2e" % (wl.name, err.max()))
        assert err.max() < TOL
    batch = lib.Batch(plans)
    rng = np.random.default_rng(77)
    for rep in range(3):
        if rep == 2:
            # new contents, same buffers: the cached graph reads them
            for (E, eta, sr, sl, V) in ins:
                V.copy_(torch.tensor(rng.uniform(-0.02, 0.02, V.numel()), device=cuda))
            eager = _eager(plans, ins)
        # the program's own eager work between replays
        x = torch.randn(1000, device=cuda).sum()
        torch.cuda.synchronize()
        outs = batch.solve(ins)
        torch.cuda.synchronize()
        for k, (o, ref) in enumerate(zip(outs, eager)):
            for a, b in zip(o, ref):
                assert np.array_equal(a.cpu().numpy(), b), "replay %d device %d" % (rep, k)
        _say("  replay %d identical to eager (%.3f), %d graph launch(es)" % (rep, float(x), batch.launches()))
        # both batches of energies of every device in one graph launch
        assert batch.launches() == 1
    for p in plans:
        assert p.status()[0] == 0
