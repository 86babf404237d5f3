"""Autotuner for the separator tree's shape: the leaf size and, on the open
slab chain (tree kind 3), the slab length.

The leaf size sets the shapes of every block the kernels see: small leaves
give many tiny fronts (latency-bound on-chip eliminations), large leaves
give fewer levels but cubic leaf work.  On the slab chain the slab length
trades the chain's depth (sequential levels, one 2w-point front each)
against the slabs' dissection (short separators with 2w-point boundaries).
The best values depend on the device's width and length and on the GPU, so
they are measured: each candidate tree is analysed, a plan is built and a
short sample of energies is solved on the GPU (timed with HIP events after
one untimed pass); the fastest candidate per energy wins.  Results are
cached per (n, width, contacts, candidates) key for the life of the
process.

Only the library's own entry points run; nothing is approximated.
"""
from __future__ import annotations

from . import Plan, analyze

_cache: dict = {}


def _key(dev, candidates):
    width = len(dev.contacts[0]) if len(dev.contacts) else 0
    return (int(dev.n), int(width), tuple(len(c) for c in dev.contacts), tuple(candidates))


def tune_leaf(dev, energies, eta, sig_r, sig_less, candidates=(8, 12, 16, 24, 32), batch=None,
              repeats=2, verbose=False, slabs=None):
    """Returns (best candidate, {candidate: ms per energy}).  Without slabs
    the candidates are leaf sizes of the nested-dissection tree; with slabs
    (a list of slab lengths) they are (slab, leaf) pairs of the open slab
    chain over dev.layers.

    dev: a device with n, rowptr, col, val, contacts, coords (and layers);
    energies: float64 tensor of sample energies on the GPU; sig_r / sig_less:
    per contact complex128 tensors [len(energies), nc, nc] on the GPU."""
    import torch
    if slabs is not None:
        candidates = tuple((sl, lf) for sl in slabs for lf in candidates)
    key = _key(dev, candidates)
    if key in _cache:
        return _cache[key]
    ne = int(energies.shape[0])
    batch = batch or ne
    times = {}
    stream = torch.cuda.current_stream(energies.device)
    for leaf in candidates:
        if slabs is None:
            sym = analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=leaf)
        else:
            sym = analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords,
                          leaf_max=leaf[1], tree_kind=3, slab=leaf[0], layers=dev.layers)
        plan = Plan(sym, max_batch=batch)
        out = plan.solve(energies, eta, sig_r, sig_less, stream=stream)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(repeats):
            plan.solve(energies, eta, sig_r, sig_less, out=out, stream=stream)
        b.record(stream)
        b.synchronize()
        times[leaf] = a.elapsed_time(b) / repeats / ne
        if verbose:
            print("  %s: %.4f ms per energy" % (leaf, times[leaf]), flush=True)
        del plan, sym, out
    best = min(times, key=times.get)
    _cache[key] = (best, times)
    return best, times


def tune_classes(devices, sample, eta, candidates=(8, 12, 16, 24, 32), verbose=False, slabs=None):
    """Tree shape per width class for a batch of devices: each class (devices
    of one contact width) is tuned on its shortest member with the sample
    energies; returns {width: leaf} (or {width: (slab, leaf)} with slabs).
    sample(dev) must return (energies, sig_r, sig_less) GPU tensors for that
    device."""
    by_width = {}
    for dev in devices:
        w = len(dev.contacts[0])
        if w not in by_width or dev.n < by_width[w].n:
            by_width[w] = dev
    out = {}
    for w, dev in sorted(by_width.items()):
        e, sr, sl = sample(dev)
        best, times = tune_leaf(dev, e, eta, sr, sl, candidates, verbose=False, slabs=slabs)
        out[w] = best
        if verbose:
            print("  width %3d (n=%d): %s  [%s]" % (
                w, dev.n, best, ", ".join("%s: %.3f" % (k, v) for k, v in sorted(times.items()))),
                flush=True)
    return out


__all__ = ["tune_leaf", "tune_classes"]
