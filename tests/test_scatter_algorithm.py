"""The G^< source with Sigma^< on every cluster, as the library organises it,
replayed on the CPU on the library's own separator tree (host-side symbolic
analysis) and checked against the dense definition.

Section 3.2 forms P_init = D^{-1} N over the fold of N = Sigma^< (G^(0))+ with
P_i = all ancestors.  The library works on frames (a cluster's points, then
its ancestors', parent first), gathers G_{B,Anc} from the lower owner's frame
rows (directly, or transposed since G^r is complex symmetric), and folds N
left-looking: each cluster pulls Psi_{d,i}^T N_{d, frame of i} from the
descendants d whose B_d meets it.  This test replays those three passes in
numpy with exact (dense) G and fold factors, and requires
P_init[i, [i, B_i]] = G^<[i, [i,B_i]] - Psi_i G^<[B_i, [i, B_i]], the identity
G^< = (I - L^T) G^< + D^{-1} L^{-1} Sigma^< G^r+ restricted to each front.
"""
import numpy as np
import pytest

from inputs import phonons, workloads


@pytest.mark.parametrize("leaf_max,coords", [(8, True), (0, True), (8, False)])
def test_frame_based_left_looking_fold_reproduces_the_source(leaf_max, coords):
    import paper_1305_1070_amd as ndg
    from oracle import definition
    wl = workloads.small_grid(20, 12, n_energies=1, noise=0.05, seed=3)
    d = wl.device
    sy = ndg.analyze(d.n, d.rowptr, d.col, d.val, d.contacts, d.coords if coords else None,
                     leaf_max=leaf_max)
    a = sy.arrays()
    perm, off, par, bptr, bidx = a["perm"], a["cl_off"], a["parent"], a["bptr"], a["bidx"]
    nc = len(par)
    s = np.diff(off)
    e = wl.energies
    sl_, sr_, _, _ = wl.self_energies(e)
    pr, pl = phonons.diagonal_self_energies(d, e, gamma0=2e-2, seed=1)
    A = definition.assemble_a(d.dense_h(), None, complex(e[0], wl.eta), d.contacts, [sl_[0], sr_[0]], pr[0])
    Ai = A[np.ix_(perm, perm)]
    sigma = pl[0][perm]                    # the phonon Sigma^< alone, internal order
    G = np.linalg.inv(Ai)
    GL = G @ np.diag(sigma) @ G.conj().T
    pts = lambda i: np.arange(off[i], off[i + 1])
    B = [bidx[bptr[i]:bptr[i + 1]] for i in range(nc)]
    # fold factors from the dense matrix in post-order
    M = Ai.copy()
    psi, ainv = {}, {}
    for i in range(nc):
        I, Bi = pts(i), B[i]
        ainv[i] = np.linalg.inv(M[np.ix_(I, I)])
        psi[i] = -ainv[i] @ M[np.ix_(I, Bi)]
        M[np.ix_(Bi, Bi)] += psi[i].T @ M[np.ix_(I, Bi)]
    # frames: chain[i] = [i, parent, ...], ao[i][t] = first frame column of chain[i][t]
    chain, ao = [], []
    for i in range(nc):
        c = [i]
        while par[c[-1]] >= 0:
            c.append(par[c[-1]])
        o = [0]
        for t in c:
            o.append(o[-1] + s[t])
        chain.append(c)
        ao.append(o)
    owner = np.zeros(d.n, int)
    for i in range(nc):
        owner[pts(i)] = i
    bpos = [[(ao[i][chain[i].index(owner[x])] + x - off[owner[x]], chain[i].index(owner[x])) for x in B[i]]
            for i in range(nc)]
    # pass 1, top-down: the G^(0) rows over each frame, gathered from the lower owner
    Gall = {}
    for i in sorted(range(nc), key=lambda i: len(chain[i])):
        g = ao[i][-1]
        X = np.zeros((len(B[i]), g), complex)
        for u, (col, au) in enumerate(bpos[i]):
            for y in range(s[i], g):
                ay = max(t for t in range(len(chain[i])) if ao[i][t] <= y)
                if ay >= au:
                    X[u, y] = Gall[chain[i][au]][col - ao[i][au], y - ao[i][au]]
                else:
                    X[u, y] = Gall[chain[i][ay]][y - ao[i][ay], col - ao[i][ay]]
        R = psi[i] @ X if len(B[i]) else np.zeros((s[i], g), complex)
        R[:, :s[i]] = G[np.ix_(pts(i), pts(i))]
        Gall[i] = R
    # pass 2, bottom-up (post-order): N_i = sigma conj(G^(0)) + sum_d Psi_{d,i}^T N_d[:, frame of i]
    feeds = {j: [] for j in range(nc)}
    for i in range(nc):
        for au in sorted({t for _, t in bpos[i]}):
            j = chain[i][au]
            um = -np.ones(s[j], int)
            for u, (col, t) in enumerate(bpos[i]):
                if t == au:
                    um[B[i][u] - off[j]] = u
            feeds[j].append((i, um, ao[i][au]))
    N = {}
    for j in range(nc):
        g = ao[j][-1]
        acc = np.zeros((s[j], g), complex)
        for dd, um, col in feeds[j]:
            Aop = np.zeros((s[j], s[dd]), complex)
            for r in range(s[j]):
                if um[r] >= 0:
                    Aop[r] = psi[dd][:, um[r]]
            acc += Aop @ N[dd][:, col:col + g]
        N[j] = sigma[pts(j)][:, None] * Gall[j].conj() + acc
    # pass 3: P_init = A_ii^{-1} N_i over the front's columns, against the identity
    worst = 0.0
    for j in range(nc):
        cols = np.concatenate([np.arange(s[j]), [c for c, _ in bpos[j]]]).astype(int)
        p0 = ainv[j] @ N[j][:, cols]
        I, F = pts(j), np.concatenate([pts(j), B[j]])
        ref = GL[np.ix_(I, F)] - (psi[j] @ GL[np.ix_(B[j], F)] if len(B[j]) else 0)
        worst = max(worst, np.max(np.abs(p0 - ref)) / np.max(np.abs(GL)))
    assert nc > 5 and max(len(c) for c in chain) > 3
    assert worst < 1e-12
