"""G^> formed in its own step and the transmission, through the C ABI
(ndg_solve_transport), against the dense oracle.

G^> = G^r Sigma^> G^r+ with Sigma^> = Sigma^< + Sigma^r - Sigma^r+ is a
further G^< pass over the same factors; it differs from the identity
G^< + G^r - G^r+ (ndg_solve's G^>) by 2 i eta diag(G^r G^r+).  The
transmission T = Tr[Gamma_0 G_01 Gamma_1 G_01+] is one more pass with the
source -i Gamma_1, read on contact 0's block.  Tolerance 1e-10: normwise per
energy for the diagonals, absolute (on max(1, T)) for T.
"""
import sys

import numpy as np
import pytest

from inputs import devices, leads, workloads

from .helpers import TOL, layer_tree, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(lib, wl, energies=None, max_batch=64, tree=None, leaf_max=8):
    import torch
    dev = wl.device
    e = wl.energies if energies is None else np.asarray(energies, np.float64)
    sl, sr, ll, lr = wl.self_energies(e)
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=leaf_max,
                      **(tree or {}))
    plan = lib.Plan(sym, max_batch=max_batch)
    cuda = torch.device("cuda:0")
    E = torch.tensor(e, device=cuda)
    srt = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (sl, sr)]
    slt = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (ll, lr)]
    gr, gl, gg, T = plan.solve_transport(E, wl.eta, srt, slt)
    gr0, gl0, gg0 = plan.solve(E, wl.eta, srt, slt)   # G^> from the identity
    torch.cuda.synchronize()
    assert plan.status()[0] == 0
    return [x.cpu().numpy() for x in (gr, gl, gg, T, gr0, gl0, gg0)], (sl, sr, ll, lr), e


@pytest.mark.parametrize("case", ["nd", "slab_chain", "slab_chain_wide"])
def test_explicit_greater_and_transmission_match_the_definition(lib, case):
    from oracle import definition
    if case == "slab_chain_wide":
        wl = workloads.small_grid(24, 80, n_energies=5, emin=0.02, emax=0.45, eta=1e-3, noise=0.03, seed=5)
    else:
        wl = workloads.small_grid(20, 12, n_energies=7, emin=0.05, emax=1.5, eta=1e-3, noise=0.05, seed=4)
    dev = wl.device
    tree = None if case == "nd" else layer_tree(dev, 3)
    # batches of 3: the extra passes' per-batch sources at every offset
    (gr, gl, gg, T, gr0, gl0, gg0), (sl, sr, ll, lr), e = _run(lib, wl, max_batch=3, tree=tree)
    _say("%s: %d energies" % (case, len(e)))
    h = dev.scipy_h()
    rgr, rgl, rgg_id = definition.diag_greens(h, None, e, wl.eta, dev.contacts, [sl, sr], [ll, lr])
    rgg = definition.diag_greater(h, None, e, wl.eta, dev.contacts, [sl, sr], [ll, lr])
    rT = definition.transmission(h, None, e, wl.eta, dev.contacts, [sl, sr])
    eg = rel_err(gg, rgg)
    er, el = rel_err(gr, rgr), rel_err(gl, rgl)
    et = np.abs(T - rT) / np.maximum(1.0, np.abs(rT))
    for k in range(len(e)):
        _say("  E=%.3f G^r %.1e G^< %.1e G^> %.1e T=%.6f err %.1e" % (e[k], er[k], el[k], eg[k], rT[k], et[k]))
    assert np.all(er < TOL) and np.all(el < TOL)
    assert np.all(eg < TOL)
    assert np.all(et < TOL)
    # the two solves agree on G^r and G^< bit for bit
    assert np.array_equal(gr, gr0) and np.array_equal(gl, gl0)
    assert np.max(rT) > 0.5


def test_explicit_minus_identity_is_the_broadening_term(lib):
    """G^r Sigma^> G^r+ - (G^< + G^r - G^r+) = 2 i eta diag(G^r G^r+): with
    eta = 2e-2 the term is well above rounding; diag(G G+) from the dense
    oracle's full G."""
    from oracle import definition
    wl = workloads.small_grid(14, 8, n_energies=4, emin=0.05, emax=0.6, eta=2e-2, noise=0.05, seed=9)
    dev = wl.device
    (gr, gl, gg, T, gr0, gl0, gg0), (sl, sr, ll, lr), e = _run(lib, wl, tree=layer_tree(wl.device, 2))
    for k in range(len(e)):
        g, _ = definition.full_greens(dev.scipy_h(), None, e[k], wl.eta, dev.contacts, [sl[k], sr[k]],
                                      [ll[k], lr[k]])
        term = 2j * wl.eta * np.sum(np.abs(g) ** 2, axis=1)
        d = gg[k] - gg0[k]
        err = np.max(np.abs(d - term)) / np.max(np.abs(gg[k]))
        _say("  E=%.3f max|term| / max|G^>| %.2e, err %.1e" % (e[k], np.max(np.abs(term)) / np.max(np.abs(gg[k])),
                                                               err))
        assert np.max(np.abs(term)) > 1e-3 * np.max(np.abs(gg[k]))
        assert err < TOL


def test_transmission_counts_open_modes(lib):
    """Uniform hard-wall waveguide at eta = 1e-9: T equals the number of open
    transverse modes (closed form)."""
    ny, nx = 24, 10
    dev = devices.fd2d(ny, nx, 0.25, 0.067, name="guide")
    t0 = dev.lead["t0"]
    _, eps = leads.transverse_modes(nx, t0)
    e = np.array([0.5, 2.0, 6.0, 15.0])
    wl = workloads.Workload("guide", dev, e, 1e-9, (0.1, 0.05), 0.025)
    (gr, gl, gg, T, *_), _, _ = _run(lib, wl, tree=layer_tree(dev, 4))
    n_open = np.array([np.sum((x > eps) & (x < eps + 4 * t0)) for x in e])
    _say("  T %s, open modes %s" % (np.round(T, 8), n_open))
    assert np.all(np.abs(T - n_open) < 1e-6)
