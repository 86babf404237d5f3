"""Density and its gradient with respect to the on-site potential, through
the C ABI: against the dense oracle (density and the oracle gradient
formula) and against central finite differences of the GPU density."""
import sys

import numpy as np
import pytest

from inputs import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup(lib, wl, leaf_max=0, max_batch=64):
    import torch
    dev = wl.device
    sl, sr, ll, lr = wl.self_energies()
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords,
                      leaf_max=leaf_max)
    plan = lib.Plan(sym, max_batch=max_batch)
    plan.enable_adjoint()
    cuda = torch.device("cuda:0")
    t = {"E": torch.tensor(wl.energies, device=cuda),
         "sig_r": [torch.from_numpy(a).to(cuda) for a in (sl, sr)],
         "sig_l": [torch.from_numpy(a).to(cuda) for a in (ll, lr)],
         "cE": torch.tensor(wl.quad_weights(), device=cuda)}
    return plan, t, (sl, sr, ll, lr)


def _density(plan, wl, t, v):
    import torch
    V = torch.tensor(v, dtype=torch.float64, device="cuda:0")
    n = plan.density(t["E"], wl.eta, t["sig_r"], t["sig_l"], t["cE"], V=V)
    torch.cuda.synchronize()
    return n.cpu().numpy()


def _vjp(plan, wl, t, v, nbar):
    import torch
    V = torch.tensor(v, dtype=torch.float64, device="cuda:0")
    nb = torch.tensor(nbar, dtype=torch.float64, device="cuda:0")
    g = plan.density_vjp(t["E"], wl.eta, t["sig_r"], t["sig_l"], t["cE"], nb, V=V)
    torch.cuda.synchronize()
    return g.cpu().numpy()


@pytest.mark.parametrize("ny,nx,leaf", [(14, 8, 8), (20, 40, 16)])
def test_density_and_vjp_match_dense_oracle(lib, ny, nx, leaf):
    """(20, 40): both contacts' 80 columns form one right-hand side (a full and
    a ragged 64-column chunk), and the 40-point separators take the tiled
    solve kernels while the leaves take the one-wavefront ones."""
    from oracle import gradient
    wl = workloads.small_grid(ny, nx, n_energies=4, emin=0.02, emax=0.3, eta=1e-3)
    dev = wl.device
    rng = np.random.default_rng(31)
    v = rng.uniform(-0.03, 0.03, dev.n)
    nbar = rng.uniform(0.5, 1.5, dev.n)
    _say("density / vjp %dx%d vs dense oracle" % (ny, nx))
    plan, t, (sl, sr, ll, lr) = _setup(lib, wl, leaf_max=leaf, max_batch=3)
    n_gpu = _density(plan, wl, t, v)
    n_ref = gradient.density(dev.scipy_h(), v, wl.energies, wl.eta, dev.contacts, [sl, sr],
                             [ll, lr], wl.quad_weights())
    assert np.max(np.abs(n_gpu - n_ref)) < 1e-10 * np.max(np.abs(n_ref))
    g_gpu = _vjp(plan, wl, t, v, nbar)
    g_ref = gradient.density_vjp(dev.scipy_h(), v, wl.energies, wl.eta, dev.contacts, [sl, sr],
                                 [ll, lr], wl.quad_weights(), nbar)
    err = np.max(np.abs(g_gpu - g_ref)) / np.max(np.abs(g_ref))
    _say("  vjp rel err %.2e" % err)
    assert err < 1e-9
    assert plan.status()[0] == 0


def test_vjp_matches_central_differences_of_gpu_density(lib):
    wl = workloads.small_grid(24, 12, n_energies=6, emin=0.01, emax=0.4, eta=1e-4)
    dev = wl.device
    rng = np.random.default_rng(5)
    v = rng.uniform(-0.02, 0.02, dev.n)
    nbar = rng.uniform(0.5, 1.5, dev.n)
    _say("vjp vs finite differences 24x12")
    plan, t, _ = _setup(lib, wl, leaf_max=16)
    g = _vjp(plan, wl, t, v, nbar)
    h = 1e-6
    for k in rng.choice(dev.n, 8, replace=False):
        vp, vm = v.copy(), v.copy()
        vp[k] += h
        vm[k] -= h
        fd = np.dot(nbar, _density(plan, wl, t, vp) - _density(plan, wl, t, vm)) / (2 * h)
        assert abs(fd - g[k]) < 1e-5 * np.max(np.abs(g)), (k, fd, g[k])


def test_autograd_function_loss_gradient(lib):
    import torch
    wl = workloads.small_grid(16, 10, n_energies=4, emin=0.02, emax=0.3, eta=1e-3)
    dev = wl.device
    rng = np.random.default_rng(9)
    v0 = rng.uniform(-0.02, 0.02, dev.n)
    w = torch.tensor(rng.uniform(0.5, 1.5, dev.n), device="cuda:0")
    plan, t, _ = _setup(lib, wl, leaf_max=10)
    target = torch.tensor(_density(plan, wl, t, rng.uniform(-0.02, 0.02, dev.n)), device="cuda:0")

    def loss_of(vnp, grad=False):
        V = torch.tensor(vnp, dtype=torch.float64, device="cuda:0", requires_grad=grad)
        n = lib.NDDensity.apply(V, plan, t["E"], wl.eta, t["sig_r"], t["sig_l"], t["cE"])
        loss = torch.sum(w * (n - target) ** 2)
        if grad:
            loss.backward()
            return loss.item(), V.grad.cpu().numpy()
        return loss.item()

    _, g = loss_of(v0, grad=True)
    h = 1e-6
    for k in [3, 50, 77, 120]:
        vp, vm = v0.copy(), v0.copy()
        vp[k] += h
        vm[k] -= h
        fd = (loss_of(vp) - loss_of(vm)) / (2 * h)
        assert abs(fd - g[k]) < 1e-5 * np.max(np.abs(g)) + 1e-14, (k, fd, g[k])


def test_adjoint_workload_512x64_fd_on_32_sites(lib):
    """The adjoint workload at full size: 512 x 64 grid, smooth +-50 meV
    potential, 256 energies, loss sum w (n - n*)^2; gradient against central
    differences (h = 1e-6 eV) of the FP64 GPU path on 32 sampled sites."""
    import torch
    wl = workloads.adjoint_device()
    dev = wl.device
    rng = np.random.default_rng(52)
    w = rng.uniform(0.5, 1.5, dev.n)
    from inputs import devices
    v_star = devices.smooth_random_potential(512, 64, 0.050, 8.0, seed=53)
    _say("adjoint workload 512x64, 256 energies")
    plan, t, _ = _setup(lib, wl, leaf_max=16, max_batch=64)
    v = wl.potential
    n_star = _density(plan, wl, t, v_star)
    n0 = _density(plan, wl, t, v)
    nbar = 2 * w * (n0 - n_star)
    g = _vjp(plan, wl, t, v, nbar)
    _say("  |g|max %.3e" % np.max(np.abs(g)))
    h = 1e-6
    loss = lambda n: np.sum(w * (n - n_star) ** 2)
    sites = rng.choice(dev.n, 32, replace=False)
    worst = 0.0
    for k in sites:
        vp, vm = v.copy(), v.copy()
        vp[k] += h
        vm[k] -= h
        fd = (loss(_density(plan, wl, t, vp)) - loss(_density(plan, wl, t, vm))) / (2 * h)
        rel = abs(fd - g[k]) / np.max(np.abs(g))
        worst = max(worst, rel)
    _say("  worst FD mismatch (relative to max|g|) %.2e" % worst)
    assert worst < 1e-5


@pytest.mark.xfail(strict=True, reason="FP32 Schur updates leave the gradient 7.4e-5 (of max|g|) from the FP64 "
                   "one and 5.6e-5 from central differences: the 1e-5 target is not met (no refinement)")
def test_adjoint_workload_mixed_products_against_fp64(lib):
    """The adjoint workload (512 x 64, 256 energies) with the fold's Schur
    updates of fronts above 64 points in complex FP32 on the matrix cores
    (NDG_MIXED; pivot inverses, Psi and the adjoint solves stay FP64): the
    gradient against the FP64 one and against central differences (h = 1e-6
    eV) of the FP64 density on 8 sampled sites, both within 1e-5 of max|g|.
    Measured: 7.4e-5 and 5.6e-5, so the target fails (strict xfail: a pass
    means the mixed path improved and this mark must go)."""
    import torch
    wl = workloads.adjoint_device()
    dev = wl.device
    rng = np.random.default_rng(52)
    w = rng.uniform(0.5, 1.5, dev.n)
    from inputs import devices
    v_star = devices.smooth_random_potential(512, 64, 0.050, 8.0, seed=53)
    _say("adjoint workload 512x64, mixed products")
    plan, t, _ = _setup(lib, wl, leaf_max=16, max_batch=64)
    v = wl.potential
    n_star = _density(plan, wl, t, v_star)
    n0 = _density(plan, wl, t, v)
    nbar = 2 * w * (n0 - n_star)
    g64 = _vjp(plan, wl, t, v, nbar)
    V = torch.tensor(v, dtype=torch.float64, device="cuda:0")
    nb = torch.tensor(nbar, dtype=torch.float64, device="cuda:0")
    g32 = plan.density_vjp(t["E"], wl.eta, t["sig_r"], t["sig_l"], t["cE"], nb, V=V,
                           prec=lib.NDG_MIXED).cpu().numpy()
    scale = np.max(np.abs(g64))
    d_mixed = np.max(np.abs(g32 - g64)) / scale
    _say("  mixed vs FP64 gradient: %.2e of max|g|" % d_mixed)
    h = 1e-6
    loss = lambda n: np.sum(w * (n - n_star) ** 2)
    worst = 0.0
    for k in rng.choice(dev.n, 8, replace=False):
        vp, vm = v.copy(), v.copy()
        vp[k] += h
        vm[k] -= h
        fd = (loss(_density(plan, wl, t, vp)) - loss(_density(plan, wl, t, vm))) / (2 * h)
        worst = max(worst, abs(fd - g32[k]) / scale)
    _say("  mixed gradient vs central differences of FP64: worst %.2e of max|g|" % worst)
    assert d_mixed < 1e-5
    assert worst < 1e-5
