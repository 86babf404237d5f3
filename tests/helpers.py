"""Shared test helpers: run the HIP path through the binding and the oracle
on the same seeded inputs."""
import numpy as np


TOL = 1e-10  # FP64 tolerance (normwise relative per energy)
CAP = 1e-6   # no bound is looser than this


def bound_vs_rgf(d_rgf):
    """Bound on the normwise error of an FP64 energy against the RGF oracle,
    given the oracle's own uncertainty d_rgf = max|x_fwd - x_rev| / max|x|
    (RGF swept from either end; the test compares with the nearer sweep).
    A result within TOL of the exact one lies within TOL + d_rgf of the
    nearer sweep.  At energies where the device itself is ill conditioned
    (a sharp resonance: both sweeps, and any FP64 method, lose digits) the
    bound follows the oracle's uncertainty, up to CAP; beyond CAP the energy
    cannot be checked in FP64 and the test fails."""
    b = TOL + 2.0 * float(d_rgf)
    assert b <= CAP, "oracle uncertainty %.1e: energy not checkable in FP64" % d_rgf
    return b


def layer_tree(dev, slab=8):
    """Keyword arguments of the open slab chain tree (kind 3) over the
    device's transport layers: every folded region holds a contact or is a
    slab of at most `slab` layers."""
    return {"tree_kind": 3, "slab": slab, "layers": dev.layers}


def rel_err(x, ref):
    """Normwise relative error max|x - ref| / max|ref| per energy (rows)."""
    x = np.atleast_2d(x)
    ref = np.atleast_2d(ref)
    den = np.maximum(np.max(np.abs(ref), axis=1), 1e-300)
    return np.max(np.abs(x - ref), axis=1) / den


def gpu_solve(ndg, wl, energies=None, max_batch=64, tree_kind=0, leaf_max=0, V=None, sym=None,
              keep_plan=False, prec=0, slab=0, layers=None):
    import torch
    dev = wl.device
    e = wl.energies if energies is None else np.asarray(energies, dtype=np.float64)
    sl, sr, ll, lr = wl.self_energies(e)
    if sym is None:
        sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords,
                          leaf_max=leaf_max, tree_kind=tree_kind, slab=slab, layers=layers)
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


def rgf_sample(args):
    """RGF oracle (both sweep directions) at one energy of a workload built
    in the worker: args = (factory name in inputs.workloads, kwargs, energy
    index).  Returns (index, (gr, gl) forward, (gr, gl) reverse)."""
    name, kwargs, idx = args
    from inputs import workloads as w
    from oracle import rgf
    wl = getattr(w, name)(**kwargs)
    d = wl.device
    e = wl.energies[[idx]]
    sl, sr, ll, lr = wl.self_energies(e)
    a = rgf.diag_greens(d.scipy_h(), None, e, wl.eta, d.layers, d.contacts, [sl, sr], [ll, lr])
    b = rgf.diag_greens(d.scipy_h(), None, e, wl.eta, d.layers[::-1], d.contacts, [sl, sr],
                        [ll, lr])
    return idx, (a[0][0], a[1][0]), (b[0][0], b[1][0])


def rgf_pool_map(jobs, workers=16):
    """Runs rgf_sample over jobs in a spawn pool, one BLAS thread each;
    results in the order of jobs."""
    import multiprocessing as mp
    import os
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        out = []
        with ctx.Pool(min(workers, len(jobs))) as pool:
            # progress lines keep a long oracle run visibly alive
            for r in pool.imap(rgf_sample, jobs, chunksize=1):
                out.append(r)
                print("  oracle %d/%d done" % (len(out), len(jobs)), flush=True)
        return out
    finally:
        for k, v in env.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
