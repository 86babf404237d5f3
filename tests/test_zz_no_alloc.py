"""ndg_density_vjp_noalloc: the density's vector-Jacobian product for callers
that cannot allocate device memory, its per-energy partials in the library's
file-scope device buffer.  Through the C ABI it must return what
ndg_density_vjp returns on the same inputs (same kernels, same order of
operations), on two calls in a row, the second with fewer energies (the
buffer keeps the last call's contents, which the call clears), and refuse a
batch whose partials do not fit the buffer."""
import sys

import numpy as np
import pytest

from inputs import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _inputs(wl, cuda):
    import torch
    sl, sr, ll, lr = wl.self_energies()
    E = torch.tensor(wl.energies, dtype=torch.float64, device=cuda)
    sig_r = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (sl, sr)]
    sig_l = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (ll, lr)]
    cE = torch.tensor(wl.quad_weights(), device=cuda)
    return E, sig_r, sig_l, cE


def test_noalloc_vjp_matches_vjp_on_two_calls(lib):
    import torch
    cuda = torch.device("cuda:0")
    wl = workloads.small_grid(30, 12, n_energies=7, emin=0.02, emax=0.4, eta=1e-4, noise=0.03,
                              seed=17)
    dev = wl.device
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=12,
                      tree_kind=3, slab=4, layers=dev.layers)
    plan = lib.Plan(sym, max_batch=4)   # 7 energies: two batches
    plan.enable_adjoint()
    E, sig_r, sig_l, cE = _inputs(wl, cuda)
    rng = np.random.default_rng(5)
    V = torch.tensor(rng.uniform(-0.02, 0.02, dev.n), device=cuda)
    nbar = torch.tensor(rng.uniform(0.5, 1.5, dev.n), device=cuda)
    out = torch.empty(dev.n, dtype=torch.float64, device=cuda)
    for ne in (7, 3):
        _say("density VJP, %d energies: ndg_density_vjp vs ndg_density_vjp_noalloc" % ne)
        args = (E[:ne].contiguous(), wl.eta, [t[:ne].contiguous() for t in sig_r],
                [t[:ne].contiguous() for t in sig_l], cE[:ne].contiguous(), nbar)
        ref = plan.density_vjp(*args, V=V)
        got = plan.density_vjp(*args, V=V, out=out, noalloc=True)
        torch.cuda.synchronize()
        assert plan.status()[0] == 0
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        err = np.max(np.abs(a - b)) / np.max(np.abs(a))
        _say("  max |noalloc - vjp| / max |vjp| = %.2e" % err)
        assert np.max(np.abs(a)) > 0
        assert err <= 1e-14


def test_noalloc_vjp_refuses_a_batch_beyond_its_buffer(lib):
    """n x min(nE, max_batch) partials above the buffer's 4 Mi doubles: a
    clear error before anything is launched."""
    import torch
    cuda = torch.device("cuda:0")
    wl = workloads.small_grid(4100, 2, n_energies=520, emin=0.02, emax=0.4, eta=1e-4, seed=3)
    dev = wl.device
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=8)
    plan = lib.Plan(sym, max_batch=520)
    plan.enable_adjoint()
    E, sig_r, sig_l, cE = _inputs(wl, cuda)
    nbar = torch.ones(dev.n, dtype=torch.float64, device=cuda)
    out = torch.empty(dev.n, dtype=torch.float64, device=cuda)
    assert dev.n * 520 > 4 << 20
    with pytest.raises(lib.NdgError) as ei:
        plan.density_vjp(E, wl.eta, sig_r, sig_l, cE, nbar, out=out, noalloc=True)
    assert "static buffer" in str(ei.value)
    _say("refused: %s" % ei.value)
