"""Host-side tests of the separator tree and symbolic analysis (no GPU):
partition rules of Section 3.2, contacts kept whole, boundary sets, and the
operation-count scaling of Section 4.1.  Also checks that the C ABI library
loads and exports every entry point include/ndnegf.h declares."""
import os
import re

import numpy as np
import pytest

import paper_1305_1070_amd as ndg
from inputs import devices, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = ndg.load()
    hdr = open(os.path.join(ROOT, "include", "ndnegf.h")).read()
    names = set(re.findall(r"\b(ndg_[a-z_]+)\s*\(", hdr))
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


def _tree(dev, **kw):
    sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, **kw)
    return sym, sym.info(), sym.arrays()


def _check_partition(dev, arr, max_s=64):
    perm, cl_off, parent, bptr, bidx = (arr[k] for k in ("perm", "cl_off", "parent", "bptr", "bidx"))
    n = dev.n
    nc = len(cl_off) - 1
    assert sorted(perm.tolist()) == list(range(n))
    iperm = np.empty(n, np.int64)
    iperm[perm] = np.arange(n)
    owner = np.empty(n, np.int64)
    for c in range(nc):
        owner[cl_off[c]:cl_off[c + 1]] = c
        assert 0 < cl_off[c + 1] - cl_off[c] <= max_s
    # ancestor sets
    anc = []
    for c in range(nc):
        a, p = set(), parent[c]
        while p >= 0:
            a.add(int(p))
            p = parent[p]
        anc.append(a)
    # rule 1: every edge joins a cluster to itself, an ancestor or a descendant
    h = dev.scipy_h().tocoo()
    for i, j in zip(h.row, h.col):
        ci, cj = owner[iperm[i]], owner[iperm[j]]
        assert ci == cj or cj in anc[ci] or ci in anc[cj]
    # contacts whole
    for cs in dev.contacts:
        assert len(set(owner[iperm[cs]].tolist())) == 1
    # boundary sets: ancestor points, ascending
    bset = []
    for c in range(nc):
        b = bidx[bptr[c]:bptr[c + 1]]
        assert np.all(np.diff(b) > 0)
        for q in b:
            assert owner[q] in anc[c]
        bset.append(set(b.tolist()))
    # and complete (Section 3.2: B_i holds the ancestor points coupled to i
    # directly or through fill passed up from its children): every coupling
    # of a point of cluster c to an ancestor's point lies in B_c ...
    for i, j in zip(h.row, h.col):
        ci, cj = owner[iperm[i]], owner[iperm[j]]
        if cj in anc[ci]:
            assert iperm[j] in bset[ci]
    for cs in dev.contacts:  # (a contact's self-energy couples all its sites)
        ic = iperm[np.asarray(cs)]
        for x in ic:
            for y in ic:
                if owner[y] in anc[owner[x]]:
                    assert y in bset[owner[x]]
    # ... and a child's boundary points outside its parent lie in the parent's B
    for c in range(nc):
        p = parent[c]
        if p >= 0:
            for q in bset[c]:
                assert owner[q] == p or q in bset[p]
    # post-order: parents after children
    for c in range(nc):
        if parent[c] >= 0:
            assert parent[c] > c


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_partition_rules_fd_grid(kind):
    dev = devices.fd2d(40, 24)
    sym, info, arr = _tree(dev, tree_kind=kind, leaf_max=16)
    _check_partition(dev, arr)


def test_partition_rules_tube_and_graph_only():
    dev = devices.zigzag_tube(12, disorder=0.1)
    _, _, arr = _tree(dev, leaf_max=24)
    _check_partition(dev, arr)
    # without coordinates: level-set separators
    sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, None, leaf_max=24)
    _check_partition(dev, sym.arrays())


def test_partition_rules_armchair_ribbon_with_vacancies():
    """The honeycomb stencil with seeded vacancies (an irregular graph), cut
    geometrically and, without coordinates, by level-set separators."""
    dev = devices.armchair_ribbon(40, 7, -2.7, disorder=0.1, vacancies=0.05)
    _, _, arr = _tree(dev, leaf_max=16)
    _check_partition(dev, arr)
    sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, None, leaf_max=16)
    _check_partition(dev, sym.arrays())


def test_rejects_nonsymmetric_h_and_overlapping_contacts():
    dev = devices.fd2d(6, 4)
    val = dev.val.copy()
    # break symmetry of one off-diagonal value
    p = next(p for p in range(dev.rowptr[0], dev.rowptr[1]) if dev.col[p] != 0)
    val[p] += 1.0
    with pytest.raises(ndg.NdgError) as ei:
        ndg.analyze(dev.n, dev.rowptr, dev.col, val, dev.contacts, dev.coords)
    assert ei.value.code == -2
    with pytest.raises(ndg.NdgError):
        ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, [dev.contacts[0], dev.contacts[0]], dev.coords)


def test_operation_count_scaling_square_and_rectangular():
    """Section 4.1: square N x N devices cost O(N^3) with nested dissection
    and O(N^4) with RGF; at fixed width the cost grows linearly in length."""
    ns = [32, 48, 64, 96, 128]
    nd_ops, rgf_ops = [], []
    for n in ns:
        dev = devices.fd2d(n, n)
        # contacts neglected (Section 4.1): analyse without contacts
        sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, [], dev.coords, leaf_max=16)
        info = sym.info()
        nd_ops.append(info["ops_total"])
        rgf_ops.append(info["ops_rgf_equiv"])
    s_nd = np.polyfit(np.log(ns), np.log(nd_ops), 1)[0]
    s_rgf = np.polyfit(np.log(ns), np.log(rgf_ops), 1)[0]
    assert 2.6 < s_nd < 3.4, s_nd
    assert abs(s_rgf - 4.0) < 0.05
    lens = [256, 512, 1024, 2048]
    ops = []
    for l in lens:
        dev = devices.fd2d(l, 32)
        sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=16)
        ops.append(sym.info()["ops_total"])
    s_len = np.polyfit(np.log(lens), np.log(ops), 1)[0]
    assert 0.85 < s_len < 1.15, s_len


def test_workspace_and_info_superlattice():
    wl = workloads.superlattice(n_energies=1)
    dev = wl.device
    sym, info, arr = _tree(dev, leaf_max=16)
    assert info["n"] == 65536 and info["max_cluster"] <= 64
    assert info["ops_total"] < 0.2 * info["ops_rgf_equiv"]
    assert 0 < info["workspace_bytes_per_energy"] < 2e9


@pytest.mark.parametrize("width", [96, 128])
def test_wide_contact_spans_a_chain_of_clusters(width):
    """A contact wider than the largest cluster (64) is split over a
    parent-child chain of clusters; the partition rules still hold."""
    dev = devices.fd2d(40, width)
    sym, info, arr = _tree(dev, leaf_max=32)
    _check_partition_chain(dev, arr)
    assert info["max_cluster"] <= 64


def _check_partition_chain(dev, arr):
    perm, cl_off, parent = arr["perm"], arr["cl_off"], arr["parent"]
    iperm = np.empty(dev.n, np.int64)
    iperm[perm] = np.arange(dev.n)
    owner = np.searchsorted(cl_off, np.arange(dev.n), side="right") - 1
    for cs in dev.contacts:
        owners = sorted(set(owner[iperm[cs]].tolist()))
        low = owners[0]
        anc = []
        p = low
        while p >= 0:
            anc.append(p)
            p = parent[p]
        assert all(o in anc for o in owners)
    h = dev.scipy_h().tocoo()
    ancs = []
    for c in range(len(cl_off) - 1):
        a, p = set(), parent[c]
        while p >= 0:
            a.add(int(p))
            p = parent[p]
        ancs.append(a)
    for i, j in zip(h.row, h.col):
        ci, cj = owner[iperm[i]], owner[iperm[j]]
        assert ci == cj or cj in ancs[ci] or ci in ancs[cj]


def _subtree_extent(dev, arr, layers):
    """Per cluster: whether its subtree holds a contact site, and how many
    transport layers its subtree's points span."""
    perm, cl_off, parent = arr["perm"], arr["cl_off"], arr["parent"]
    nc = len(parent)
    layer_of = np.empty(dev.n, np.int64)
    for q, L in enumerate(layers):
        layer_of[L] = q
    is_contact = np.zeros(dev.n, bool)
    for cs in dev.contacts:
        is_contact[cs] = True
    lo = np.full(nc, 1 << 40)
    hi = np.full(nc, -1)
    has = np.zeros(nc, bool)
    for c in range(nc):  # post-order: children first
        sites = perm[cl_off[c]:cl_off[c + 1]]
        lo[c] = min(lo[c], layer_of[sites].min())
        hi[c] = max(hi[c], layer_of[sites].max())
        has[c] |= is_contact[sites].any()
        p = parent[c]
        if p >= 0:
            lo[p] = min(lo[p], lo[c])
            hi[p] = max(hi[p], hi[c])
            has[p] |= has[c]
    return has, hi - lo + 1


@pytest.mark.parametrize("width,slab", [(24, 4), (24, -1), (64, 8), (96, 8), (128, 12)])
def test_open_slab_chain_tree(width, slab):
    """Tree kind 3: every folded region either holds a contact (open) or is
    a slab of at most `slab` layers; separator layers up to 128 points stay
    one cluster; the partition rules hold."""
    dev = devices.fd2d(60, width)
    sym, info, arr = _tree(dev, tree_kind=3, slab=slab, leaf_max=16, layers=dev.layers)
    _check_partition(dev, arr, max_s=128)
    has, span = _subtree_extent(dev, arr, dev.layers)
    assert np.all(has | (span <= max(slab, 0)))
    assert info["max_cluster"] == width
    # the root is a middle layer; both contacts' clusters are chain ends
    root = int(np.nonzero(arr["parent"] < 0)[0][0])
    sites = arr["perm"][arr["cl_off"][root]:arr["cl_off"][root + 1]]
    assert set(sites.tolist()) == set(dev.layers[30].tolist())
    if slab < 0:
        assert info["nclusters"] == 60 and info["max_height"] == 31


def test_open_slab_chain_tube_cells():
    """The tube's 40-atom cells as layers: with no slabs (every cell a
    separator) the tree is the layer chain of Section 3.2, Fig. 6, rooted in
    the middle cell, so every folded region holds a contact."""
    dev = devices.zigzag_tube(16, disorder=0.1)
    sym, info, arr = _tree(dev, tree_kind=3, slab=-1, layers=dev.layers)
    _check_partition(dev, arr)
    has, _ = _subtree_extent(dev, arr, dev.layers)
    assert has.all() and info["nclusters"] == 16


def test_open_slab_chain_rejects_non_tridiagonal_layers():
    dev = devices.fd2d(10, 6)
    bad = [np.concatenate([dev.layers[0], dev.layers[2]]), dev.layers[1]] + list(dev.layers[3:])
    with pytest.raises(ndg.NdgError):
        ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, tree_kind=3,
                    layers=bad)


def _recount(dev, arr):
    """Flops per launch group recomputed from the tree arrays (Section 4.1's
    convention, 8 flops per complex multiply-add)."""
    perm, cl_off, parent, height, bptr = (arr[k] for k in ("perm", "cl_off", "parent", "height", "bptr"))
    nc = len(parent)
    s = np.diff(cl_off).astype(float)
    b = np.diff(bptr).astype(float)
    kids = np.zeros(nc, int)
    for p in parent:
        if p >= 0:
            kids[p] += 1
    iperm = np.empty(dev.n, int)
    iperm[perm] = np.arange(dev.n)
    owner = np.searchsorted(cl_off, np.arange(dev.n), side="right") - 1
    chain_of = []
    for cs in dev.contacts:
        ch, k = set(), int(owner[iperm[cs]].min())
        while k >= 0:
            ch.add(k)
            k = parent[k]
        chain_of.append(ch)
    out = {}

    def add(name, h, q, v):
        out[(name, h, q)] = out.get((name, h, q), 0.0) + v

    for k in range(nc):
        sk, bk, h = s[k], b[k], int(height[k])
        f = sk + bk
        q = (0 if f <= 32 else 1 if f <= 48 else 2) if f <= 64 else \
            (3 if sk <= 16 else 4 if sk <= 32 else 5 if sk <= 64 else 6)
        if f <= 64:
            add("k_fold_small", h, q, 8 * (sk ** 3 + sk * sk * bk + sk * bk * bk))
            diag = kids[k] == 0 and not any(k in c for c in chain_of)
            for nm in ("k_extract_small(G)", "k_extract_small(P)"):
                add(nm, h, q, 8 * (sk * bk * bk + (sk * bk if diag else sk * sk * bk)))
        else:
            add("k_factor", h, q, 8 * sk ** 3)
            add("k_psi", h, q, 8 * sk * sk * bk)
            add("k_update", h, q, 8 * sk * bk * bk)
            for nm in ("k_down_off(G)", "k_down_off(P)"):
                add(nm, h, q, 8 * sk * bk * bk)
            for nm in ("k_down_diag(G)", "k_down_diag(P)"):
                add(nm, h, q, 8 * sk * sk * bk)
        for c, cs in zip(chain_of, dev.contacts):
            if k in c:
                sc = len(cs)
                add("k_chain_fwd", h, 0, 8 * (sk * bk * sc + sk * sk * sc))
                add("k_chain_back", h, 0, 8 * (sk * bk * sc + sk * sc * f))
                add("k_chain_t", 0, 0, 8 * sk * sc * sc)
    return out


@pytest.mark.parametrize("case", ["nd", "slab_chain_wide", "tube_cells"])
def test_cost_table_sums_to_op_count_and_recounts(case):
    """The per-launch-group cost table the profiler credits each launch with
    (one group per kernel, height and size class) sums to 8 x ops_total and
    equals a recount from the tree arrays."""
    if case == "nd":
        dev = devices.fd2d(60, 40)
        sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=16)
    elif case == "slab_chain_wide":
        dev = devices.fd2d(50, 96)
        sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, leaf_max=16,
                          tree_kind=3, slab=6, layers=dev.layers)
    else:
        dev = devices.zigzag_tube(20, disorder=0.1)
        sym = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords, tree_kind=3,
                          slab=-1, layers=dev.layers)
    costs = sym.costs()
    info = sym.info()
    total = sum(c["flops"] for c in costs)
    assert total == pytest.approx(8 * info["ops_total"], rel=1e-12)
    got = {(c["name"], c["height"], c["size_class"]): c["flops"] for c in costs if c["flops"] > 0}
    ref = {k: v for k, v in _recount(dev, sym.arrays()).items() if v > 0}
    assert set(got) == set(ref)
    for key, v in ref.items():
        assert got[key] == pytest.approx(v, rel=1e-12), key
    # several size classes share a height (one launch each)
    assert len({(n, h) for n, h, _ in got}) < len(got) or case == "tube_cells"
