"""Newton step of the Schroedinger-Poisson problem through the C ABI
(ndg_poisson_newton_step) against the oracle's dense step.

F(V) = K V - beta (n(V) - n_D), J = K - beta dn/dV.  The library solves
J delta = -F by conjugate gradients, applying dn/dV through the density's
vector-Jacobian product (exact in equilibrium, where dn/dV is symmetric);
the oracle assembles dn/dV densely and solves directly.  8 x 6 grid, both
contacts at 2.2 eV, eta = 0 in the device, 31 energies over the occupied
band.  Tolerance: 1e-9 relative on delta (the CG stops at 1e-13).
"""
import sys

import numpy as np
import pytest

from inputs import devices, leads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem():
    import scipy.sparse as sp
    from oracle import gradient
    dev = devices.fd2d(8, 6)
    e = np.linspace(1.7, 2.6, 31)
    w = np.full(e.size, e[1] - e[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    cE = w / (2 * np.pi)
    sig = leads.contact_self_energies(dev, e, 1e-7, (2.2, 2.2), 0.025)
    h = dev.scipy_h()
    a = (h != 0).astype(float).toarray()
    np.fill_diagonal(a, 0.0)
    K = 0.05 * (np.diag(a.sum(1)) - a + 0.5 * np.eye(dev.n))
    sl_, sr_, ll_, lr_ = sig
    n0 = gradient.density(h, None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_], cE)
    return dev, e, cE, sig, K, sp.csr_matrix(K), 1.0, 1.3 * n0


def _gpu(lib, dev, e, cE, sig, Kcsr, beta, nd):
    import torch
    cuda = torch.device("cuda:0")
    sym = lib.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=8)
    plan = lib.Plan(sym, max_batch=16)
    plan.enable_adjoint()
    sl_, sr_, ll_, lr_ = sig
    t = dict(
        E=torch.tensor(e, device=cuda), cE=torch.tensor(cE, device=cuda),
        sr=[torch.from_numpy(np.ascontiguousarray(x)).to(cuda) for x in (sl_, sr_)],
        sl=[torch.from_numpy(np.ascontiguousarray(x)).to(cuda) for x in (ll_, lr_)],
        rp=torch.tensor(Kcsr.indptr.astype(np.int64), device=cuda),
        col=torch.tensor(Kcsr.indices.astype(np.int32), device=cuda),
        val=torch.tensor(Kcsr.data.astype(np.float64), device=cuda),
        nd=torch.tensor(nd, device=cuda))

    def step(v):
        V = torch.tensor(v, device=cuda)
        d, fn, it, res = plan.poisson_newton_step(t["E"], 0.0, t["sr"], t["sl"], t["cE"], V, t["rp"], t["col"],
                                                  t["val"], beta, t["nd"], cg_tol=1e-13, cg_max_iter=300)
        torch.cuda.synchronize()
        return d.cpu().numpy(), fn, it, res
    return step


def test_newton_step_matches_oracle(lib):
    from oracle import poisson
    dev, e, cE, sig, K, Kcsr, beta, nd = _problem()
    sl_, sr_, ll_, lr_ = sig
    step = _gpu(lib, dev, e, cE, sig, Kcsr, beta, nd)
    rng = np.random.default_rng(5)
    for v in (np.zeros(dev.n), rng.uniform(-0.05, 0.05, dev.n)):
        d, fn, it, res = step(v)
        dref, fref = poisson.newton_step(dev.scipy_h(), v, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_], cE, K,
                                         beta, nd)
        err = np.max(np.abs(d - dref)) / np.max(np.abs(dref))
        _say("newton step: |F| gpu %.6e oracle %.6e, cg %d iterations (rel %.1e), delta err %.2e"
             % (fn, np.linalg.norm(fref), it, res, err))
        assert abs(fn - np.linalg.norm(fref)) <= 1e-10 * np.linalg.norm(fref)
        assert res <= 1e-13 and err < 1e-9


def test_newton_iterations_converge(lib):
    """V <- V + delta from V = 0: the residual falls below 1e-10 of the
    first within six steps, and the last steps square it."""
    dev, e, cE, sig, K, Kcsr, beta, nd = _problem()
    step = _gpu(lib, dev, e, cE, sig, Kcsr, beta, nd)
    v = np.zeros(dev.n)
    norms = []
    for _ in range(6):
        d, fn, it, res = step(v)
        norms.append(fn)
        v = v + d
    _say("newton |F|: " + " ".join("%.2e" % x for x in norms))
    assert norms[-1] < 1e-10 * norms[0]


def test_newton_step_reports_indefinite_jacobian(lib):
    """K = 0 and beta = -1 make J = dn/dV, negative definite: the first
    conjugate-gradient step finds p^T J p <= 0 and returns NDG_ENOTSPD (a
    condition set from the host; every kernel exits normally)."""
    import scipy.sparse as sp
    dev, e, cE, sig, K, Kcsr, beta, nd = _problem()
    # one explicit zero entry (an empty CSR would pass null index arrays)
    zero = sp.csr_matrix((np.zeros(1), np.zeros(1, np.int32), np.r_[0, np.ones(dev.n, np.int64)]),
                         shape=(dev.n, dev.n))
    assert zero.nnz == 1
    step = _gpu(lib, dev, e, cE, sig, zero, -1.0, nd)
    with pytest.raises(lib.NdgError) as ei:
        step(np.zeros(dev.n))
    assert ei.value.code == -8
    _say("indefinite Jacobian reported: %s" % ei.value)
