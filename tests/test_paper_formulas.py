"""The paper's printed block formulas, checked against the dense definition.

These pin the readings of the paper that the HIP path is built on:
  * Section 3.1 (three clusters L, R, S): Schur complement, G^r_SS, G^r_LS,
    G^r_LL, G^<_SS, G^<_LS and G^<_LL.  The printed G^<_LL carries a minus
    in front of A_LL^{-1} A_LS (G^<_LS)+; the identity G^< = (I - L^T) G^< +
    D^{-1} L^{-1} Sigma^< G^r+ with G^<_SL = -(G^<_LS)+ gives a plus, and so do
    the multilevel step 4 and the appendix.  The test shows the plus is right
    and the minus is not.
  * The appendix (three-level tree, clusters 1, 2, 4 leaves, 3 on level 2,
    5 the root; 1 and 4 dense): every printed block of A^(1), A^(2), G^(2..0),
    N^(1..2), P^(2..0), with N = Sigma^< (G^(0))+ (the appendix writes
    (G^<)+; G^(0) is what Section 3.2 step 1 uses) and with the right-hand
    sides of the P^(0) updates read as the previous-level values.
Inputs: random complex-symmetric A with the appendix's block sparsity and a
random block-diagonal skew-Hermitian, purely imaginary Sigma^<.
"""
import numpy as np
import pytest

RNG = np.random.default_rng(1305)


def _sym(m):
    return 0.5 * (m + m.T)


def _rand_c(r, c):
    return RNG.standard_normal((r, c)) + 1j * RNG.standard_normal((r, c))


def _blocks(sizes):
    off = np.concatenate([[0], np.cumsum(sizes)])
    return [slice(off[i], off[i + 1]) for i in range(len(sizes))], off[-1]


def _make(sizes, couplings, seed_shift=4.0):
    """Random complex-symmetric A with nonzero off-diagonal blocks only at
    `couplings` (pairs, 0-based), and Sigma^< = i * (real symmetric) per block."""
    sl, n = _blocks(sizes)
    a = np.zeros((n, n), np.complex128)
    for i, s in enumerate(sl):
        a[s, s] = _sym(_rand_c(sizes[i], sizes[i])) + seed_shift * np.eye(sizes[i])
    for i, j in couplings:
        b = _rand_c(sizes[i], sizes[j])
        a[sl[i], sl[j]] = b
        a[sl[j], sl[i]] = b.T
    sig = np.zeros((n, n), np.complex128)
    for i, s in enumerate(sl):
        q = RNG.standard_normal((sizes[i], sizes[i]))
        sig[s, s] = 1j * (q @ q.T)
    return a, sig, sl


def _close(x, y, tol=1e-10):
    return np.max(np.abs(x - y)) <= tol * max(1.0, np.max(np.abs(y)))


def test_three_cluster_formulas_and_sign_of_gless_ll():
    sizes = [5, 4, 3]  # L, R, S
    a, sig, (L, R, S) = _make(sizes, [(0, 2), (1, 2)])
    g = np.linalg.inv(a)
    gl = g @ sig @ g.conj().T
    inv = np.linalg.inv
    all_, arr, ass = a[L, L], a[R, R], a[S, S]
    als, ars = a[L, S], a[R, S]
    hat = ass - als.T @ inv(all_) @ als - ars.T @ inv(arr) @ ars
    gss = inv(hat)
    assert _close(gss, g[S, S])
    gls = -inv(all_) @ als @ gss
    assert _close(gls, g[L, S])
    gll = inv(all_) + inv(all_) @ als @ gss @ als.T @ inv(all_)
    assert _close(gll, g[L, L])
    # lesser
    s_ll, s_rr, s_ss = sig[L, L], sig[R, R], sig[S, S]
    g_sl, g_sr = g[S, L], g[S, R]
    gl_ss = gss @ (s_ss @ gss.conj().T - als.T @ inv(all_) @ s_ll @ g_sl.conj().T
                   - ars.T @ inv(arr) @ s_rr @ g_sr.conj().T)
    assert _close(gl_ss, gl[S, S])
    gl_ls = -inv(all_) @ als @ gl_ss + inv(all_) @ s_ll @ g_sl.conj().T
    assert _close(gl_ls, gl[L, S])
    plus = inv(all_) @ s_ll @ g[L, L].conj().T + inv(all_) @ als @ gl_ls.conj().T
    minus = inv(all_) @ s_ll @ g[L, L].conj().T - inv(all_) @ als @ gl_ls.conj().T
    assert _close(plus, gl[L, L])
    assert not _close(minus, gl[L, L], tol=1e-3)


@pytest.fixture(scope="module")
def appendix():
    sizes = [6, 5, 4, 6, 4]  # clusters 1..5 -> indices 0..4; 1 and 4 are the dense contacts
    # couplings of the appendix's A: 13, 15, 23, 25, 35, 45
    a, sig, sl = _make(sizes, [(0, 2), (0, 4), (1, 2), (1, 4), (2, 4), (3, 4)])
    # Sigma^< only on the contact clusters 1 and 4 (plus a general case below)
    return a, sig, sl


def test_appendix_three_level_gr(appendix):
    a, _, sl = appendix
    inv = np.linalg.inv
    B = lambda i, j: a[sl[i - 1], sl[j - 1]]
    g = np.linalg.inv(a)
    G = lambda i, j: g[sl[i - 1], sl[j - 1]]
    # A^(1)
    a33 = B(3, 3) - B(1, 3).T @ inv(B(1, 1)) @ B(1, 3) - B(2, 3).T @ inv(B(2, 2)) @ B(2, 3)
    a35 = B(3, 5) - B(1, 3).T @ inv(B(1, 1)) @ B(1, 5) - B(2, 3).T @ inv(B(2, 2)) @ B(2, 5)
    a55 = (B(5, 5) - B(1, 5).T @ inv(B(1, 1)) @ B(1, 5) - B(2, 5).T @ inv(B(2, 2)) @ B(2, 5)
           - B(4, 5).T @ inv(B(4, 4)) @ B(4, 5))
    # A^(2)
    a55_2 = a55 - a35.T @ inv(a33) @ a35
    # G^(2): root block and G^(1)
    g55 = inv(a55_2)
    assert _close(g55, G(5, 5))
    psi35 = -inv(a33) @ a35
    g35 = psi35 @ g55
    g33 = inv(a33) + psi35 @ g35.T
    assert _close(g35, G(3, 5)) and _close(g33, G(3, 3))
    # G^(0): region 4
    g45 = -inv(B(4, 4)) @ B(4, 5) @ g55
    g44 = inv(B(4, 4)) - inv(B(4, 4)) @ B(4, 5) @ g45.T
    assert _close(g45, G(4, 5)) and _close(g44, G(4, 4))
    # region 1 and 2
    for r in (1, 2):
        air = inv(B(r, r))
        gr5 = -air @ B(r, 5) @ g55 - air @ B(r, 3) @ g35
        gr3 = -air @ B(r, 3) @ g33 - air @ B(r, 5) @ g35.T
        grr = air - air @ B(r, 3) @ gr3.T - air @ B(r, 5) @ gr5.T
        assert _close(gr5, G(r, 5)) and _close(gr3, G(r, 3)) and _close(grr, G(r, r))


@pytest.mark.parametrize("sigma_on", ["contacts", "all"])
def test_appendix_three_level_gless(appendix, sigma_on):
    a, sig_all, sl = appendix
    sig = sig_all.copy()
    if sigma_on == "contacts":
        for i in (1, 2, 4):  # clusters 2, 3, 5 carry no Sigma^<
            sig[sl[i], sl[i]] = 0
    inv = np.linalg.inv
    B = lambda i, j: a[sl[i - 1], sl[j - 1]]
    g = np.linalg.inv(a)
    gl = g @ sig @ g.conj().T
    G = lambda i, j: g[sl[i - 1], sl[j - 1]]
    GL = lambda i, j: gl[sl[i - 1], sl[j - 1]]
    S = lambda i: sig[sl[i - 1], sl[i - 1]]
    a33 = B(3, 3) - B(1, 3).T @ inv(B(1, 1)) @ B(1, 3) - B(2, 3).T @ inv(B(2, 2)) @ B(2, 3)
    a35 = B(3, 5) - B(1, 3).T @ inv(B(1, 1)) @ B(1, 5) - B(2, 3).T @ inv(B(2, 2)) @ B(2, 5)
    a55 = (B(5, 5) - B(1, 5).T @ inv(B(1, 1)) @ B(1, 5) - B(2, 5).T @ inv(B(2, 2)) @ B(2, 5)
           - B(4, 5).T @ inv(B(4, 4)) @ B(4, 5))
    a55_2 = a55 - a35.T @ inv(a33) @ a35
    # N = Sigma^< (G^(0))+ on the stored pattern of G^(0) (G^(0) entries = G^r entries)
    N = {}
    for i, j in [(1, 1), (1, 3), (1, 5), (2, 2), (2, 3), (2, 5), (3, 3), (3, 5), (4, 4), (4, 5),
                 (5, 5)]:
        N[(i, j)] = S(i) @ G(j, i).conj().T   # (G+)_{ij} = (G_{ji})+
    for i, j in [(3, 1), (3, 2), (5, 1), (5, 2), (5, 3), (5, 4)]:
        N[(i, j)] = S(i) @ G(j, i).conj().T
    # N^(1)
    n33 = N[(3, 3)] - B(1, 3).T @ inv(B(1, 1)) @ N[(1, 3)] - B(2, 3).T @ inv(B(2, 2)) @ N[(2, 3)]
    n55 = (N[(5, 5)] - B(1, 5).T @ inv(B(1, 1)) @ N[(1, 5)] - B(2, 5).T @ inv(B(2, 2)) @ N[(2, 5)]
           - B(4, 5).T @ inv(B(4, 4)) @ N[(4, 5)])
    n35 = N[(3, 5)] - B(1, 3).T @ inv(B(1, 1)) @ N[(1, 5)] - B(2, 3).T @ inv(B(2, 2)) @ N[(2, 5)]
    # N^(2)
    n55_2 = n55 - a35.T @ inv(a33) @ n35
    # P^(2) = D^{-1} N on the needed blocks
    p55 = inv(a55_2) @ n55_2
    p35 = inv(a33) @ n35
    p33 = inv(a33) @ n33
    assert _close(p55, GL(5, 5))
    # P^(1)
    p35_1 = p35 - inv(a33) @ a35 @ p55
    p53_1 = -p35_1.conj().T
    p33_1 = p33 - inv(a33) @ a35 @ p53_1
    assert _close(p35_1, GL(3, 5)) and _close(p53_1, GL(5, 3)) and _close(p33_1, GL(3, 3))
    # P^(0): region 4
    p45 = inv(B(4, 4)) @ N[(4, 5)] - inv(B(4, 4)) @ B(4, 5) @ p55
    p44 = inv(B(4, 4)) @ N[(4, 4)] + inv(B(4, 4)) @ B(4, 5) @ p45.conj().T
    assert _close(p45, GL(4, 5)) and _close(p44, GL(4, 4))
    for r in (1, 2):
        air = inv(B(r, r))
        pr5 = air @ N[(r, 5)] - air @ B(r, 5) @ p55 - air @ B(r, 3) @ p35_1
        pr3 = air @ N[(r, 3)] - air @ B(r, 3) @ p33_1 + air @ B(r, 5) @ p35_1.conj().T
        prr = air @ N[(r, r)] + air @ B(r, 3) @ pr3.conj().T + air @ B(r, 5) @ pr5.conj().T
        assert _close(pr5, GL(r, 5)) and _close(pr3, GL(r, 3)) and _close(prr, GL(r, r))


# ---------------------------------------------------------------------------
# Section 3.2's multilevel algorithms on a tree where a cluster has an
# ancestor it is not coupled to, with Sigma^< on every cluster (the diagonal
# phonon case): P_i is the set of ALL ancestors of i (the paper's
# definition), and the N fold needs every (cluster, ancestor) block of
# G^(0).  Restricting P_i to the ancestors coupled to i after fill (which is
# exact for G^r, where Psi_ij = 0 for the others) loses terms of N.
# ---------------------------------------------------------------------------

def _chain7():
    """Seven clusters in a line, 1-2-3-4-5-6-7 (0-based 0..6): leaves 1, 3,
    5, 7 (level 1), separators 2 and 6 (level 2), root 4 (level 3).  Cluster
    1 couples to 2 only: its ancestors are {2, 4}, but only 2 is coupled to
    it, before or after fill."""
    sizes = [4, 3, 4, 3, 4, 3, 4]
    a, sig, sl = _make(sizes, [(k, k + 1) for k in range(6)])
    parent = [1, 3, 1, -1, 5, 3, 5]
    level = [1, 2, 1, 3, 1, 2, 1]
    return a, sig, sl, parent, level


def _ancestors(parent, i):
    out = []
    while parent[i] >= 0:
        i = parent[i]
        out.append(i)
    return out


def _multilevel(a, sig, sl, parent, level, ancestor_sets):
    """G^r and G^< blocks by the four steps of Section 3.2, with the given
    ancestor set per cluster standing for P_i.  Returns dicts of blocks."""
    inv = np.linalg.inv
    nl = max(level)
    A = {(i, j): a[sl[i], sl[j]].copy() for i in range(len(sl)) for j in range(len(sl))}
    on = lambda l: [i for i in range(len(sl)) if level[i] == l]
    P = ancestor_sets
    # fold: A_jk += Psi_ij^T A_ik for j, k in P_i
    psi = {}
    for l in range(1, nl):
        for i in on(l):
            ainv = inv(A[(i, i)])
            for j in P[i]:
                psi[(i, j)] = -ainv @ A[(i, j)]
            for j in P[i]:
                for k in P[i]:
                    A[(j, k)] = A[(j, k)] + psi[(i, j)].T @ A[(i, k)]
    root = on(nl)[0]
    # G^r extraction
    G = {(root, root): inv(A[(root, root)])}
    for l in range(nl - 1, 0, -1):
        for i in on(l):
            for j in P[i]:
                G[(i, j)] = sum(psi[(i, k)] @ G[(k, j)] for k in P[i])
            for j in P[i]:
                G[(j, i)] = G[(i, j)].T
            G[(i, i)] = inv(A[(i, i)]) + sum(psi[(i, j)] @ G[(j, i)] for j in P[i])
    # step 1: N = Sigma^< (G^(0))+ on the blocks (i, k), k in {i} and P_i
    S = lambda i: sig[sl[i], sl[i]]
    N = {}
    for i in range(len(sl)):
        for k in [i] + list(P[i]):
            N[(i, k)] = S(i) @ G[(k, i)].conj().T
    # step 2: N_jk += Psi_ij^T N_ik for j, k in P_i
    for l in range(1, nl):
        for i in on(l):
            for j in P[i]:
                for k in P[i]:
                    N[(j, k)] = N.get((j, k), 0) + psi[(i, j)].T @ N[(i, k)]
    # step 3: P = D^{-1} N on the same blocks
    Pl = {(i, k): inv(A[(i, i)]) @ N[(i, k)] for (i, k) in N
          if k == i or k in P[i]}
    # step 4: extraction
    for l in range(nl - 1, 0, -1):
        for i in on(l):
            for j in P[i]:
                Pl[(i, j)] = Pl[(i, j)] + sum(psi[(i, k)] @ Pl[(k, j)] for k in P[i])
            for j in P[i]:
                Pl[(j, i)] = -Pl[(i, j)].conj().T
            Pl[(i, i)] = Pl[(i, i)] + sum(psi[(i, j)] @ Pl[(j, i)] for j in P[i])
    return G, Pl


@pytest.mark.parametrize("sigma_on", ["ends", "all"])
def test_multilevel_needs_all_ancestors_for_gless(sigma_on):
    a, sig, sl, parent, level = _chain7()
    if sigma_on == "ends":
        for i in range(1, 6):  # Sigma^< on the two end clusters only (contacts)
            sig[sl[i], sl[i]] = 0
    g = np.linalg.inv(a)
    gl = g @ sig @ g.conj().T
    anc = [_ancestors(parent, i) for i in range(7)]
    G, Pl = _multilevel(a, sig, sl, parent, level, anc)
    for i in range(7):
        assert _close(G[(i, i)], g[sl[i], sl[i]])
        assert _close(Pl[(i, i)], gl[sl[i], sl[i]])
    # the coupled ancestors only: cluster 1 (index 0) loses ancestor 4 (3),
    # cluster 7 (index 6) likewise; G^r is unchanged, G^< is not
    coupled = [a_ for a_ in anc]
    coupled[0] = [1]
    coupled[6] = [5]
    G2, Pl2 = _multilevel(a, sig, sl, parent, level, coupled)
    for i in range(7):
        assert _close(G2[(i, i)], g[sl[i], sl[i]])
    assert not all(_close(Pl2[(i, i)], gl[sl[i], sl[i]]) for i in range(7))
