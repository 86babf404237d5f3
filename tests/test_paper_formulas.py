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
