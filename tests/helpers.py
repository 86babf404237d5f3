"""Shared test helpers: run the HIP path through the binding and the oracle
on the same seeded inputs."""
import numpy as np


def rel_err(x, ref):
    """Normwise relative error max|x - ref| / max|ref| per energy (rows)."""
    x = np.atleast_2d(x)
    ref = np.atleast_2d(ref)
    den = np.maximum(np.max(np.abs(ref), axis=1), 1e-300)
    return np.max(np.abs(x - ref), axis=1) / den


def gpu_solve(ndg, wl, energies=None, max_batch=64, tree_kind=0, leaf_max=0, V=None, sym=None,
              keep_plan=False, prec=0):
    import torch
    dev = wl.device
    e = wl.energies if energies is None else np.asarray(energies, dtype=np.float64)
    sl, sr, ll, lr = wl.self_energies(e)
    if sym is None:
        sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords,
                          leaf_max=leaf_max, tree_kind=tree_kind)
    plan = ndg.Plan(sym, max_batch=max_batch)
    cuda = torch.device("cuda:0")
    E = torch.tensor(e, dtype=torch.float64, device=cuda)
    sig_r = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (sl, sr)]
    sig_l = [torch.from_numpy(np.ascontiguousarray(a)).to(cuda) for a in (ll, lr)]
    Vt = None
    if V is not None:
        Vt = torch.tensor(np.asarray(V, dtype=np.float64), device=cuda)
    growth = torch.zeros(len(e), dtype=torch.float64, device=cuda)
    gr, gl, gg = plan.solve(E, wl.eta, sig_r, sig_l, V=Vt, growth=growth, prec=prec)
    torch.cuda.synchronize()
    out = (gr.cpu().numpy(), gl.cpu().numpy(), gg.cpu().numpy(), growth.cpu().numpy())
    status = plan.status()
    if keep_plan:
        return out, status, plan, sym
    return out, status


def oracle_dense(wl, energies=None, V=None):
    from oracle import definition
    dev = wl.device
    e = wl.energies if energies is None else np.asarray(energies, dtype=np.float64)
    sl, sr, ll, lr = wl.self_energies(e)
    return definition.diag_greens(dev.scipy_h(), V, e, wl.eta, dev.contacts, [sl, sr], [ll, lr])


def oracle_rgf(wl, energies=None, V=None):
    from oracle import rgf
    dev = wl.device
    e = wl.energies if energies is None else np.asarray(energies, dtype=np.float64)
    sl, sr, ll, lr = wl.self_energies(e)
    return rgf.diag_greens(dev.scipy_h(), V, e, wl.eta, dev.layers, dev.contacts, [sl, sr],
                           [ll, lr])
