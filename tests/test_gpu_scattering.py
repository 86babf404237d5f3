"""Parity of the phonon-scattering solve (diagonal Sigma^r_ph, Sigma^<_ph)
through the C ABI with the dense definition of the oracle.

The library forms the G^< source of every cluster by the four steps of
Section 3.2 with P_i = all ancestors (the rows of G^(0) over every
(cluster, ancestor) pair, the fold of N = Sigma^< (G^(0))+, D^{-1} N), then
extracts G^< as without phonons.  Tolerance: 1e-10 normwise relative per
energy (FP64) where the fold is well conditioned, as for ndg_solve.  At the
superlattice's size, where the dense oracle is out of reach, the
fluctuation-dissipation identity G^< = -f (G^r - G^r*) checks the path on
every diagonal entry (equilibrium, eta = 0 in the device).
"""
import sys

import numpy as np
import pytest

from inputs import devices, leads, phonons, workloads

from .helpers import TOL, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(ndg, dev, e, eta, sig, pr, pl, max_batch=64, tree_kind=0, leaf_max=0, enable=True,
         slab=0):
    import torch
    sl_, sr_, ll_, lr_ = sig
    sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords,
                      leaf_max=leaf_max, tree_kind=tree_kind, slab=slab,
                      layers=dev.layers if tree_kind == 3 else None)
    plan = ndg.Plan(sym, max_batch=max_batch)
    if enable:
        plan.enable_scattering()
    cuda = torch.device("cuda:0")
    E = torch.tensor(np.asarray(e, np.float64), device=cuda)
    sr = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (sl_, sr_)]
    sl = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (ll_, lr_)]
    prt = None if pr is None else torch.from_numpy(np.ascontiguousarray(pr)).to(cuda)
    plt = None if pl is None else torch.from_numpy(np.ascontiguousarray(pl)).to(cuda)
    growth = torch.zeros(len(e), dtype=torch.float64, device=cuda)
    gr, gl, gg = plan.solve_scattering(E, eta, sr, sl, prt, plt, growth=growth)
    torch.cuda.synchronize()
    code, energy, cluster = plan.status()
    assert code == 0, (code, energy, cluster)
    return gr.cpu().numpy(), gl.cpu().numpy(), gg.cpu().numpy(), growth.cpu().numpy(), plan


def _oracle(dev, e, eta, sig, pr, pl):
    from oracle import definition
    sl_, sr_, ll_, lr_ = sig
    return definition.diag_greens(dev.scipy_h(), None, e, eta, dev.contacts, [sl_, sr_], [ll_, lr_],
                                  pr, pl)


def _check(out, ref, what):
    growth = out[3]
    er = rel_err(out[0], ref[0])
    el = rel_err(out[1], ref[1])
    scale = np.maximum(np.max(np.abs(ref[0]), axis=-1), np.max(np.abs(ref[1]), axis=-1))
    eg = np.max(np.abs(out[2] - ref[2]), axis=-1) / scale
    bad = []
    for k in range(len(growth)):
        _say("  %s energy %d growth %.3e errs %.2e %.2e %.2e" % (what, k, growth[k], er[k], el[k], eg[k]))
        if not max(er[k], el[k], eg[k]) < TOL:
            bad.append(k)
    assert not bad, bad


@pytest.mark.parametrize("tree_kind,leaf_max", [(0, 0), (0, 8), (1, 0), (2, 0), (3, 8)])
def test_scattering_small_grid_matches_definition(lib, tree_kind, leaf_max):
    wl = workloads.small_grid(20, 12, n_energies=5, emin=0.02, emax=0.4, eta=1e-3, noise=0.05, seed=4)
    e = wl.energies
    sig = wl.self_energies(e)
    pr, pl = phonons.diagonal_self_energies(wl.device, e, gamma0=1e-2, seed=2)
    _say("scattering 20x12 tree_kind=%d leaf_max=%d" % (tree_kind, leaf_max))
    out = _run(lib, wl.device, e, wl.eta, sig, pr, pl, tree_kind=tree_kind, leaf_max=leaf_max)
    ref = _oracle(wl.device, e, wl.eta, sig, pr, pl)
    _check(out, ref, "tree %d leaf %d" % (tree_kind, leaf_max))
    # the phonon source is not negligible here
    ref0 = _oracle(wl.device, e, wl.eta, sig, pr, None)
    assert np.max(rel_err(ref0[1], ref[1])) > 1e-3


def test_scattering_batches_and_ragged_tail(lib):
    """7 energies through a plan of 3 (batches 3, 3, 1); larger fronts
    (32 x 16, default leaves) that take the tiled kernels."""
    wl = workloads.small_grid(32, 16, n_energies=7, emin=0.05, emax=0.35, eta=1e-3, noise=0.03, seed=8)
    e = wl.energies
    sig = wl.self_energies(e)
    pr, pl = phonons.diagonal_self_energies(wl.device, e, gamma0=5e-3, seed=5)
    _say("scattering 32x16 max_batch=3")
    out = _run(lib, wl.device, e, wl.eta, sig, pr, pl, max_batch=3)
    ref = _oracle(wl.device, e, wl.eta, sig, pr, pl)
    _check(out, ref, "32x16")


def test_scattering_wide_contacts(lib):
    """Contacts of 80 sites span a parent-child chain of clusters: their part
    of the source comes from the chains and is added to the phonon part."""
    wl = workloads.small_grid(10, 80, n_energies=3, emin=0.05, emax=0.3, eta=1e-3, noise=0.03, seed=9)
    e = wl.energies
    sig = wl.self_energies(e)
    pr, pl = phonons.diagonal_self_energies(wl.device, e, gamma0=1e-2, seed=6)
    _say("scattering 10x80 (wide contacts)")
    out = _run(lib, wl.device, e, wl.eta, sig, pr, pl)
    ref = _oracle(wl.device, e, wl.eta, sig, pr, pl)
    _check(out, ref, "10x80")


def test_scattering_retarded_only_and_none(lib):
    """Sigma^r_ph alone needs no scattering workspace (the contacts' chains
    carry the whole source); with neither it equals ndg_solve."""
    import torch
    from .helpers import gpu_solve
    wl = workloads.small_grid(16, 10, n_energies=3, emin=0.05, emax=0.3, eta=1e-3, noise=0.05, seed=6)
    e = wl.energies
    sig = wl.self_energies(e)
    pr, _ = phonons.diagonal_self_energies(wl.device, e, gamma0=1e-2, seed=3)
    _say("scattering Sigma^r_ph only")
    out = _run(lib, wl.device, e, wl.eta, sig, pr, None, enable=False)
    ref = _oracle(wl.device, e, wl.eta, sig, pr, None)
    _check(out, ref, "r only")
    _say("scattering without phonon terms vs ndg_solve")
    out0 = _run(lib, wl.device, e, wl.eta, sig, None, None, enable=False)
    plain, _ = gpu_solve(lib, wl)
    for a, b in zip(out0[:3], plain[:3]):
        assert np.array_equal(a, b)
    torch.cuda.synchronize()


def test_scattering_needs_enable(lib):
    import torch
    wl = workloads.small_grid(8, 6, n_energies=2, eta=1e-3)
    e = wl.energies
    sig = wl.self_energies(e)
    pr, pl = phonons.diagonal_self_energies(wl.device, e, seed=1)
    with pytest.raises(lib.NdgError):
        _run(lib, wl.device, e, wl.eta, sig, pr, pl, enable=False)
    torch.cuda.synchronize()


@pytest.mark.parametrize("nt", [256, 1024])
def test_scattering_superlattice_equilibrium_identity(lib, nt):
    """Superlattice nt x 64 (the full-size geometry at nt = 1024), one
    chemical potential for the leads and every phonon site, eta = 0 in the
    device: diag G^< = -f (G^r - conj(G^r)) on all sites."""
    wl = workloads.superlattice(n_transport=nt, n_energies=4)
    dev = wl.device
    e = np.array([0.03, 0.08, 0.12, 0.21])
    mu = (0.1, 0.1)
    sig = leads.contact_self_energies(dev, e, 1e-6, mu, wl.kt)
    pr, pl = phonons.diagonal_self_energies(dev, e, gamma0=5e-3, mu=mu, seed=11, equilibrium=True)
    _say("scattering superlattice %dx64 equilibrium" % nt)
    gr, gl, gg, growth, plan = _run(lib, dev, e, 0.0, sig, pr, pl, max_batch=4, leaf_max=20,
                                    tree_kind=3, slab=12)
    _say("  scatter workspace %.1f MB per energy" % (plan.info()["scatter_bytes_per_energy"] / 1e6))
    f = leads.fermi(e, mu[0], wl.kt)[:, None]
    rhs = -f * (gr - gr.conj())
    err = np.max(np.abs(gl - rhs), axis=1) / np.max(np.abs(rhs), axis=1)
    for k in range(len(e)):
        _say("  E=%.3f growth %.3e err %.2e" % (e[k], growth[k], err[k]))
        assert err[k] < TOL
    # G^> = G^< + G^r - G^r* = (1 - f)(G^r - G^r*) in equilibrium
    assert np.max(np.abs(gg - (1 - f) * (gr - gr.conj()))) <= 1e-9 * np.max(np.abs(gr))


def _scba_gpu(ndg, dev, e, eta, sig, d0, mix, tol, max_iter, leaf_max=0, max_batch=64):
    import torch
    sl_, sr_, ll_, lr_ = sig
    sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=leaf_max)
    plan = ndg.Plan(sym, max_batch=max_batch)
    plan.enable_scattering()
    cuda = torch.device("cuda:0")
    E = torch.tensor(np.asarray(e, np.float64), device=cuda)
    sr = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (sl_, sr_)]
    sl = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (ll_, lr_)]
    gr, gl, gg, spr, spl, it, res = plan.scba(E, eta, sr, sl, d0, mix, tol, max_iter)
    torch.cuda.synchronize()
    assert plan.status()[0] == 0
    return (gr.cpu().numpy(), gl.cpu().numpy(), gg.cpu().numpy(), spr.cpu().numpy(), spl.cpu().numpy(),
            it, res)


def test_scba_matches_oracle_loop(lib):
    """The Born loop on the GPU against the oracle's loop: same iterations,
    the same self-energies and Green's functions (both iterate the same
    contraction from zero; FP64 differences of one solve stay at 1e-15)."""
    from oracle import scba
    dev = devices.fd2d(16, 8)
    e = np.linspace(1.2, 1.8, 5)              # first transverse band of the 8-wide lead
    mu = (1.5, 1.4)
    sig = leads.contact_self_energies(dev, e, 1e-6, mu, 0.025)
    sl_, sr_, ll_, lr_ = sig
    _say("scba 16x8 d0=0.1")
    out = _scba_gpu(lib, dev, e, 1e-6, sig, 0.1, 0.7, 1e-10, 60, leaf_max=8)
    ref = scba.scba(dev.scipy_h(), None, e, 1e-6, dev.contacts, [sl_, sr_], [ll_, lr_], 0.1, 0.7, 1e-10, 60)
    _say("  iterations gpu %d oracle %d, residual gpu %.2e oracle %.2e" % (out[5], ref[5], out[6], ref[6]))
    assert out[5] == ref[5] and out[6] < 1e-10
    for k, name in ((0, "Gr"), (1, "Gless"), (3, "Sigma^r_ph"), (4, "Sigma^<_ph")):
        err = np.max(rel_err(out[k], ref[k]))
        _say("  %s max rel err %.2e" % (name, err))
        assert err < 1e-10, name


def test_scba_superlattice_equilibrium(lib):
    """Superlattice 256 x 64, leads at one chemical potential, eta = 0 in
    the device: every Born iterate keeps the fluctuation-dissipation pairs,
    so the converged G^< = -f (G^r - G^r*) and
    Sigma^<_ph = -f (Sigma^r_ph - Sigma^r_ph*) on every site."""
    wl = workloads.superlattice(n_transport=256, n_energies=4)
    dev = wl.device
    e = np.array([0.04, 0.09, 0.15, 0.22])
    mu = (0.1, 0.1)
    sig = leads.contact_self_energies(dev, e, 1e-6, mu, wl.kt)
    _say("scba superlattice 256x64 equilibrium")
    gr, gl, gg, spr, spl, it, res = _scba_gpu(lib, dev, e, 0.0, sig, 0.05, 0.8, 1e-9, 80, leaf_max=20,
                                              max_batch=4)
    _say("  iterations %d residual %.2e max |Sigma^r_ph| %.3e" % (it, res, np.abs(spr).max()))
    assert res < 1e-9 and it > 2
    f = leads.fermi(e, mu[0], wl.kt)[:, None]
    assert np.max(rel_err(gl, -f * (gr - gr.conj()))) < 1e-9
    assert np.max(rel_err(spl, -f * (spr - spr.conj()))) < 1e-9


def _currents(ndg, dev, e, eta, sig, pr, pl, leaf_max=0, enable=True):
    import torch
    sl_, sr_, ll_, lr_ = sig
    sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=leaf_max)
    plan = ndg.Plan(sym, max_batch=64)
    if enable:
        plan.enable_scattering()
    cuda = torch.device("cuda:0")
    E = torch.tensor(np.asarray(e, np.float64), device=cuda)
    sr = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (sl_, sr_)]
    sl = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (ll_, lr_)]
    prt = None if pr is None else torch.from_numpy(np.ascontiguousarray(pr)).to(cuda)
    plt = None if pl is None else torch.from_numpy(np.ascontiguousarray(pl)).to(cuda)
    cur = torch.full((len(e), 2), float("nan"), dtype=torch.float64, device=cuda)
    plan.solve_scattering(E, eta, sr, sl, prt, plt, current=cur)
    torch.cuda.synchronize()
    assert plan.status()[0] == 0
    return cur.cpu().numpy()


@pytest.mark.parametrize("phonon", [False, True])
def test_terminal_currents_match_oracle(lib, phonon):
    """Current spectral density per contact against the oracle's trace
    formula, ballistic (where it is the Landauer current) and with fixed
    phonon self-energies on every site."""
    from oracle import definition
    dev = devices.fd2d(16, 8)
    e = np.linspace(1.2, 1.8, 6)
    mu = (1.55, 1.35)
    sig = leads.contact_self_energies(dev, e, 1e-6, mu, 0.025)
    sl_, sr_, ll_, lr_ = sig
    pr, pl = (phonons.diagonal_self_energies(dev, e, gamma0=2e-2, mu=mu, seed=8) if phonon
              else (None, None))
    _say("currents 16x8 phonon=%s" % phonon)
    cur = _currents(lib, dev, e, 1e-6, sig, pr, pl, leaf_max=8, enable=phonon)
    ref = definition.terminal_currents(dev.scipy_h(), None, e, 1e-6, dev.contacts, [sl_, sr_], [ll_, lr_],
                                       pr, pl)
    err = np.max(np.abs(cur - ref), axis=1) / np.max(np.abs(ref), axis=1)
    _say("  currents %s\n  max rel err %.2e" % (np.array2string(cur[:, 0], precision=4), err.max()))
    assert np.all(err < 1e-10)


def test_terminal_currents_wide_contacts(lib):
    """80-site contacts span a parent-child chain of clusters: the contact
    block is read across the chain's stored rows."""
    from oracle import definition
    wl = workloads.small_grid(10, 80, n_energies=3, emin=0.05, emax=0.3, eta=1e-3, noise=0.03, seed=9)
    e = wl.energies
    sig = wl.self_energies(e)
    sl_, sr_, ll_, lr_ = sig
    _say("currents 10x80 (wide contacts)")
    cur = _currents(lib, wl.device, e, wl.eta, sig, None, None, enable=False)
    ref = definition.terminal_currents(wl.device.scipy_h(), None, e, wl.eta, wl.device.contacts,
                                       [sl_, sr_], [ll_, lr_])
    err = np.max(np.abs(cur - ref), axis=1) / np.max(np.abs(ref), axis=1)
    _say("  max rel err %.2e" % err.max())
    assert np.all(err < 1e-10)


def test_scba_conserves_current_superlattice(lib):
    """Superlattice 256 x 64 under bias, eta = 0 in the device: at the Born
    fixed point of local elastic scattering no current goes into the
    phonons, so i_L + i_R = 0 per energy, while the current differs from the
    ballistic one."""
    import torch
    wl = workloads.superlattice(n_transport=256, n_energies=4)
    dev = wl.device
    e = np.array([0.06, 0.09, 0.12, 0.15])
    sig = leads.contact_self_energies(dev, e, 1e-6, wl.mu, wl.kt)
    sl_, sr_, ll_, lr_ = sig
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=20)
    plan = lib.Plan(sym, max_batch=4)
    plan.enable_scattering()
    cuda = torch.device("cuda:0")
    E = torch.tensor(e, device=cuda)
    sr = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (sl_, sr_)]
    sl = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (ll_, lr_)]
    cur = torch.zeros((len(e), 2), dtype=torch.float64, device=cuda)
    _say("scba superlattice 256x64 under bias")
    *_, it, res = plan.scba(E, 0.0, sr, sl, 0.05, 0.8, 1e-9, 100, current=cur)
    bal = torch.zeros_like(cur)
    plan.solve_scattering(E, 0.0, sr, sl, current=bal)
    torch.cuda.synchronize()
    c, b = cur.cpu().numpy(), bal.cpu().numpy()
    _say("  iterations %d residual %.2e\n  i_L %s\n  i_R %s\n  ballistic %s" % (
        it, res, np.array2string(c[:, 0], precision=5), np.array2string(c[:, 1], precision=5),
        np.array2string(b[:, 0], precision=5)))
    assert res < 1e-9
    # against the largest current (at 0.06 eV the current sits in a minigap)
    assert np.max(np.abs(c[:, 0] + c[:, 1])) <= 1e-7 * np.max(np.abs(c[:, 0]))
    assert np.max(np.abs(b[:, 0] + b[:, 1])) <= 1e-7 * np.max(np.abs(b[:, 0]))
    assert np.max(np.abs(c[:, 0] - b[:, 0])) > 1e-2 * np.max(np.abs(b[:, 0]))


def test_scattering_deep_tree_refused_and_empty_calls(lib):
    """A layer chain of 80 layers (tree depth 80) would need every later
    layer in each frame: enable_scattering refuses it (NDG_EINVAL) before
    allocating.  nE = 0 returns at once."""
    import torch
    dev = devices.fd2d(80, 4)
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, tree_kind=1)
    plan = lib.Plan(sym, max_batch=2)
    with pytest.raises(lib.NdgError) as ei:
        plan.enable_scattering()
    assert ei.value.code == -1
    assert plan.info()["scatter_bytes_per_energy"] == 0
    wl = workloads.small_grid(8, 6, n_energies=2, eta=1e-3)
    sym2 = lib.analyze(wl.device.n, wl.device.rowptr, wl.device.col, wl.device.val, wl.device.contacts,
                       wl.device.coords)
    plan2 = lib.Plan(sym2, max_batch=2)
    plan2.enable_scattering()
    cuda = torch.device("cuda:0")
    n = wl.device.n
    E = torch.zeros(0, dtype=torch.float64, device=cuda)
    z = [torch.zeros((0, 6, 6), dtype=torch.complex128, device=cuda) for _ in range(2)]
    ph = torch.zeros((0, n), dtype=torch.complex128, device=cuda)
    gr, gl, gg = plan2.solve_scattering(E, 1e-3, z, z, ph, ph)
    assert gr.shape == (0, n)
    *_, it, res = plan2.scba(E, 1e-3, z, z, 0.1)
    assert it == 0 and res == 0.0
    torch.cuda.synchronize()


def test_scba_ragged_batches_match_oracle(lib):
    """The Born loop over 5 energies in batches of 2 (2, 2, 1): every
    iteration solves all energies before the mixing step."""
    from oracle import scba
    dev = devices.fd2d(12, 8)
    e = np.linspace(1.25, 1.75, 5)
    sig = leads.contact_self_energies(dev, e, 1e-6, (1.5, 1.4), 0.025)
    sl_, sr_, ll_, lr_ = sig
    _say("scba 12x8 batches of 2")
    out = _scba_gpu(lib, dev, e, 1e-6, sig, 0.1, 0.7, 1e-10, 60, leaf_max=8, max_batch=2)
    ref = scba.scba(dev.scipy_h(), None, e, 1e-6, dev.contacts, [sl_, sr_], [ll_, lr_], 0.1, 0.7, 1e-10, 60)
    _say("  iterations gpu %d oracle %d" % (out[5], ref[5]))
    assert out[5] == ref[5]
    for k in (0, 1, 3, 4):
        assert np.max(rel_err(out[k], ref[k])) < 1e-10


def test_scattering_tiny_device(lib):
    """A 3 x 4 device (12 sites, the root possibly a leaf with no
    ancestors): phonon solve and currents against the definition."""
    from oracle import definition
    wl = workloads.small_grid(3, 4, n_energies=3, emin=0.05, emax=0.3, eta=1e-3, noise=0.05, seed=13)
    dev = wl.device
    e = wl.energies
    sig = wl.self_energies(e)
    sl_, sr_, ll_, lr_ = sig
    pr, pl = phonons.diagonal_self_energies(dev, e, gamma0=2e-2, seed=9)
    info = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords).info()
    _say("tiny device: %d clusters, %d levels" % (info["nclusters"], info["max_height"]))
    out = _run(lib, dev, e, wl.eta, sig, pr, pl)
    _check(out, _oracle(dev, e, wl.eta, sig, pr, pl), "3x4")
    cur = _currents(lib, dev, e, wl.eta, sig, pr, pl)
    ref = definition.terminal_currents(dev.scipy_h(), None, e, wl.eta, dev.contacts, [sl_, sr_], [ll_, lr_],
                                       pr, pl)
    assert np.max(np.abs(cur - ref)) <= 1e-10 * np.max(np.abs(ref))
