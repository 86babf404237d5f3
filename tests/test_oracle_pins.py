"""Pins of the CPU oracle against facts other than itself.

Each test checks the oracle (definition.py, rgf.py, brute.py, gradient.py)
against something the mathematics or the physics fixes independently:
50-digit brute force, closed forms of the uniform hard-wall waveguide
(written here from the characteristic roots of the 1-D chain, not from the
square-root form the input generator uses), unit transmission per open mode,
the Bloch band count of the pristine tube, the Keldysh identities, and
finite differences.
"""
import numpy as np
import pytest

from inputs import devices, leads, phonons, workloads
from oracle import brute, definition, gradient, poisson, rgf, scba

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _problem(wl, energies=None):
    e = wl.energies if energies is None else np.asarray(energies)
    sl, sr, ll, lr = wl.self_energies(e)
    return e, [sl, sr], [ll, lr]


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


# ---------------------------------------------------------------------------
# brute force (no LAPACK) <-> dense <-> RGF
# ---------------------------------------------------------------------------

def test_dense_matches_mpmath_bruteforce():
    wl = workloads.small_grid(6, 4, n_energies=2, emin=0.05, emax=0.25, eta=1e-3, noise=0.05, seed=11)
    e, sr, sl = _problem(wl)
    h = wl.device.dense_h()
    dgr, dgl, _ = definition.diag_greens(h, None, e, wl.eta, wl.device.contacts, sr, sl)
    for k in range(len(e)):
        bgr, bgl = brute.diag_greens(h, None, e[k], wl.eta, wl.device.contacts,
                                     [s[k] for s in sr], [s[k] for s in sl])
        assert _rel(dgr[k], bgr) < 1e-11
        assert _rel(dgl[k], bgl) < 1e-10


def test_rgf_matches_mpmath_bruteforce_directly():
    wl = workloads.small_grid(7, 3, n_energies=2, emin=0.02, emax=0.2, eta=1e-4, noise=0.1, seed=5)
    e, sr, sl = _problem(wl)
    h = wl.device.dense_h()
    rgr, rgl, _ = rgf.diag_greens(wl.device.scipy_h(), None, e, wl.eta, wl.device.layers,
                                  wl.device.contacts, sr, sl)
    for k in range(len(e)):
        bgr, bgl = brute.diag_greens(h, None, e[k], wl.eta, wl.device.contacts,
                                     [s[k] for s in sr], [s[k] for s in sl])
        assert _rel(rgr[k], bgr) < 1e-11
        assert _rel(rgl[k], bgl) < 1e-10


def test_rgf_matches_dense_fd_with_potential():
    v = np.random.default_rng(3).uniform(-0.1, 0.1, 20 * 12)
    dev = devices.fd2d(20, 12, potential=None)
    wl = workloads.Workload("t", dev, np.linspace(0.0, 0.4, 3), 1e-6, (0.1, 0.05), 0.025)
    e, sr, sl = _problem(wl)
    dgr, dgl, dgg = definition.diag_greens(dev.scipy_h(), v, e, wl.eta, dev.contacts, sr, sl)
    rgr, rgl, rgg = rgf.diag_greens(dev.scipy_h(), v, e, wl.eta, dev.layers, dev.contacts, sr, sl)
    assert _rel(rgr, dgr) < 1e-10
    assert _rel(rgl, dgl) < 1e-9
    assert _rel(rgg, dgg) < 1e-9


def test_rgf_matches_dense_tube():
    wl = workloads.nanotube(n_cells=4, n_energies=3)
    e, sr, sl = _problem(wl, [-0.8, 0.1, 0.9])
    dev = wl.device
    dgr, dgl, _ = definition.diag_greens(dev.scipy_h(), None, e, wl.eta, dev.contacts, sr, sl)
    rgr, rgl, _ = rgf.diag_greens(dev.scipy_h(), None, e, wl.eta, dev.layers, dev.contacts, sr, sl)
    assert _rel(rgr, dgr) < 1e-9
    assert _rel(rgl, dgl) < 1e-8


# ---------------------------------------------------------------------------
# closed forms of the uniform hard-wall waveguide
# ---------------------------------------------------------------------------

def _chain_root(z, eps_long, t0):
    """Decaying root lambda (|lambda| < 1) of t0 l^2 + (z - eps_long) l + t0 = 0."""
    r = np.roots([t0, z - eps_long, t0])
    return r[np.argmin(np.abs(r))]


def _waveguide_closed_form(ny, nx, t0, z, f_l, f_r):
    """diag G^r and diag G^< of an ny x nx uniform waveguide between two
    identical semi-infinite leads, mode by mode.

    Mode m: transverse energy eps_m, longitudinal chain on-site 2 t0 + eps_m,
    hopping -t0.  Infinite chain: G(y, y') = C lambda^|y - y'| with
    C = 1 / (z - eps' + 2 t0 lambda).  Lead self-energy of the mode is
    -t0 lambda, Gamma_m = 2 t0 Im(lambda)."""
    x = np.arange(1, nx + 1)
    gr = np.zeros((ny, nx), np.complex128)
    gl = np.zeros((ny, nx), np.complex128)
    y = np.arange(ny)
    for m in range(1, nx + 1):
        phi2 = (2.0 / (nx + 1)) * np.sin(m * np.pi * x / (nx + 1)) ** 2
        eps_long = 2 * t0 + 2 * t0 * (1 - np.cos(m * np.pi / (nx + 1)))
        lam = _chain_root(z, eps_long, t0)
        c = 1.0 / (z - eps_long + 2 * t0 * lam)
        gam = 2 * t0 * lam.imag
        gr += np.outer(np.full(ny, c), phi2)
        occ = f_l * gam * np.abs(c * lam ** y) ** 2 + f_r * gam * np.abs(c * lam ** (ny - 1 - y)) ** 2
        gl += 1j * np.outer(occ, phi2)
    return gr.ravel(), gl.ravel()


@pytest.mark.parametrize("eta", [1e-6, 1e-2])
def test_dense_matches_waveguide_closed_form(eta):
    ny, nx = 16, 8
    wl = workloads.uniform_waveguide(ny, nx, n_energies=5, emax=0.6, eta=eta)
    e, sr, sl = _problem(wl)
    dgr, dgl, _ = definition.diag_greens(wl.device.scipy_h(), None, e, eta, wl.device.contacts, sr, sl)
    t0 = wl.device.lead["t0"]
    for k in range(len(e)):
        f_l = leads.fermi(e[k], wl.mu[0], wl.kt)
        f_r = leads.fermi(e[k], wl.mu[1], wl.kt)
        cgr, cgl = _waveguide_closed_form(ny, nx, t0, complex(e[k], eta), f_l, f_r)
        assert _rel(dgr[k], cgr) < 1e-10
        assert _rel(dgl[k], cgl) < 1e-9


def test_rgf_matches_waveguide_closed_form_cfg_shape():
    """64 x 32 uniform waveguide at its 16 energies (the small FP64 workload)."""
    wl = workloads.uniform_waveguide()
    e, sr, sl = _problem(wl)
    rgr, rgl, _ = rgf.diag_greens(wl.device.scipy_h(), None, e, wl.eta, wl.device.layers,
                                  wl.device.contacts, sr, sl)
    t0 = wl.device.lead["t0"]
    for k in range(len(e)):
        f_l = leads.fermi(e[k], wl.mu[0], wl.kt)
        f_r = leads.fermi(e[k], wl.mu[1], wl.kt)
        cgr, cgl = _waveguide_closed_form(64, 32, t0, complex(e[k], wl.eta), f_l, f_r)
        assert _rel(rgr[k], cgr) < 1e-9
        if np.max(np.abs(cgl)) > 0:
            assert _rel(rgl[k], cgl) < 1e-8


def test_unit_transmission_per_open_mode():
    ny, nx = 10, 6
    wl = workloads.uniform_waveguide(ny, nx, n_energies=1, eta=1e-9)
    t0 = wl.device.lead["t0"]
    _, eps = leads.transverse_modes(nx, t0)
    for e in [0.5, 2.0, 6.0, 15.0]:
        s = leads.fd_lead_sigma(complex(e, 1e-9), nx, t0)
        g, _ = definition.full_greens(wl.device.scipy_h(), None, e, 1e-9, wl.device.contacts,
                                      [s, s], [0 * s, 0 * s])
        l0, ln = wl.device.contacts
        g1n = g[np.ix_(l0, ln)]
        gam = leads.gamma(s)
        t = np.trace(gam @ g1n @ gam @ g1n.conj().T).real
        n_open = int(np.sum((e > eps) & (e < eps + 4 * t0)))
        assert abs(t - n_open) < 1e-6


# ---------------------------------------------------------------------------
# Keldysh identities
# ---------------------------------------------------------------------------

def test_lesser_is_skew_hermitian_and_occupation_nonnegative():
    wl = workloads.small_grid(8, 5, n_energies=3, eta=1e-3, noise=0.05, seed=2)
    e, sr, sl = _problem(wl)
    for k in range(len(e)):
        g, gl = definition.full_greens(wl.device.scipy_h(), None, e[k], wl.eta, wl.device.contacts,
                                       [s[k] for s in sr], [s[k] for s in sl])
        assert np.max(np.abs(gl + gl.conj().T)) < 1e-12 * np.max(np.abs(gl))
        d = np.diag(gl)
        assert np.max(np.abs(d.real)) < 1e-12 * np.max(np.abs(d))
        assert np.min((-1j * d).real) > -1e-14


def test_spectral_identity_with_eta_broadening():
    """G^r - G^r+ = -i G^r (Gamma_L + Gamma_R + 2 eta I) G^r+."""
    wl = workloads.small_grid(9, 4, n_energies=2, eta=1e-2, noise=0.05, seed=9)
    e, sr, _ = _problem(wl)
    n = wl.device.n
    for k in range(len(e)):
        g, _ = definition.full_greens(wl.device.scipy_h(), None, e[k], wl.eta, wl.device.contacts,
                                      [s[k] for s in sr], [0 * s[k] for s in sr])
        gam = np.zeros((n, n), np.complex128)
        for sites, s in zip(wl.device.contacts, sr):
            gam[np.ix_(sites, sites)] += leads.gamma(s[k])
        gam += 2 * wl.eta * np.eye(n)
        lhs = g - g.conj().T
        rhs = -1j * g @ gam @ g.conj().T
        assert _rel(lhs, rhs) < 1e-11


def test_equilibrium_lesser():
    """mu_L = mu_R: G^< = -f (G^r - G^r+) - 2 i eta f G^r G^r+."""
    dev = devices.fd2d(8, 4)
    wl = workloads.Workload("eq", dev, np.array([0.05, 0.2]), 1e-2, (0.1, 0.1), 0.025)
    e, sr, sl = _problem(wl)
    for k in range(len(e)):
        g, gl = definition.full_greens(dev.scipy_h(), None, e[k], wl.eta, dev.contacts,
                                       [s[k] for s in sr], [s[k] for s in sl])
        f = leads.fermi(e[k], 0.1, 0.025)
        rhs = -f * (g - g.conj().T) - 2j * wl.eta * f * g @ g.conj().T
        assert _rel(gl, rhs) < 1e-11


def test_density_is_occupied_lead_spectral_weight_in_equilibrium():
    """definition.density's sign and factor -i, pinned by the equilibrium
    identity above: -i G^<_ii = f (A_ii - 2 eta (G G^+)_ii) with
    A = -2 Im G^r, i.e. f (G Gamma_leads G^+)_ii, so the density with
    weights c_E is sum_E c_E f(E) (G Gamma_leads G^+)_ii >= 0."""
    dev = devices.fd2d(8, 4)
    wl = workloads.Workload("eq", dev, np.array([0.05, 0.1, 0.2]), 1e-2, (0.1, 0.1), 0.025)
    e, sr, sl = _problem(wl)
    c_e = np.array([0.3, 0.5, 0.2])
    dgl, ref = [], np.zeros(dev.n)
    for k in range(len(e)):
        g, gl = definition.full_greens(dev.scipy_h(), None, e[k], wl.eta, dev.contacts,
                                       [s[k] for s in sr], [s[k] for s in sl])
        dgl.append(np.diag(gl))
        f = leads.fermi(e[k], 0.1, 0.025)
        a = -2.0 * np.imag(np.diag(g))
        ref += c_e[k] * f * (a - 2.0 * wl.eta * np.real(np.diag(g @ g.conj().T)))
    n = definition.density(np.array(dgl), c_e)
    assert np.all(n > 0)
    assert _rel(n, ref) < 1e-11


# ---------------------------------------------------------------------------
# diagonal phonon self-energies (Sigma^r_Phonon of equation defineA, diagonal
# as Section 1 takes it; its lesser part adds to Sigma^<)
# ---------------------------------------------------------------------------

def test_phonon_inputs_are_physical_self_energies():
    """The generator's Sigma^<_ph is anti-Hermitian on the diagonal (purely
    imaginary, Im >= 0: in-scattering), Im Sigma^r_ph < 0 (retarded), and in
    equilibrium mode Sigma^<_ph = -f (Sigma^r_ph - conj(Sigma^r_ph))
    exactly; the same seed gives the same arrays."""
    dev = devices.fd2d(10, 6)
    e = np.linspace(0.0, 0.5, 7)
    pr, pl = phonons.diagonal_self_energies(dev, e, gamma0=1e-2, seed=4)
    assert np.all(pl.real == 0) and np.all(pl.imag >= 0)
    assert np.all(pr.imag < 0)
    pr2, pl2 = phonons.diagonal_self_energies(dev, e, gamma0=1e-2, seed=4)
    assert np.array_equal(pr, pr2) and np.array_equal(pl, pl2)
    qr, ql = phonons.diagonal_self_energies(dev, e, gamma0=1e-2, mu=(0.2, 0.2), seed=4, equilibrium=True)
    f = leads.fermi(e, 0.2, 0.025)[:, None]
    assert np.max(np.abs(ql + f * (qr - qr.conj()))) <= 1e-15 * np.max(np.abs(ql))


def test_phonon_dense_matches_mpmath_bruteforce():
    wl = workloads.small_grid(5, 4, n_energies=2, emin=0.05, emax=0.25, eta=1e-3, noise=0.05, seed=12)
    e, sr, sl = _problem(wl)
    pr, pl = phonons.diagonal_self_energies(wl.device, e, gamma0=2e-2, seed=3)
    h = wl.device.dense_h()
    dgr, dgl, _ = definition.diag_greens(h, None, e, wl.eta, wl.device.contacts, sr, sl, pr, pl)
    for k in range(len(e)):
        bgr, bgl = brute.diag_greens(h, None, e[k], wl.eta, wl.device.contacts,
                                     [s[k] for s in sr], [s[k] for s in sl],
                                     sig_r_ph=pr[k], sig_less_ph=pl[k])
        assert _rel(dgr[k], bgr) < 1e-11
        assert _rel(dgl[k], bgl) < 1e-10
    # the phonon terms are not negligible at this size
    dgr0, dgl0, _ = definition.diag_greens(h, None, e, wl.eta, wl.device.contacts, sr, sl)
    assert _rel(dgr0, dgr) > 1e-3 and _rel(dgl0, dgl) > 1e-3


@pytest.mark.parametrize("gamma", [1e-3, 2e-2])
def test_phonon_uniform_broadening_matches_waveguide_closed_form(gamma):
    """Sigma^r_ph = -i gamma / 2 on every site (Sigma^<_ph = 0) turns the
    device's z = E + i eta into E + i (eta + gamma / 2); with the leads taken
    at that z too, the closed form of the infinite waveguide holds there."""
    ny, nx, eta = 16, 8, 1e-6
    wl = workloads.uniform_waveguide(ny, nx, n_energies=4, emax=0.6, eta=eta)
    e = wl.energies
    eta2 = eta + 0.5 * gamma
    sl_, sr_, ll_, lr_ = leads.contact_self_energies(wl.device, e, eta2, wl.mu, wl.kt)
    n = wl.device.n
    pr = np.full((len(e), n), -0.5j * gamma)
    pl = np.zeros((len(e), n), np.complex128)
    dgr, dgl, _ = definition.diag_greens(wl.device.scipy_h(), None, e, eta, wl.device.contacts,
                                         [sl_, sr_], [ll_, lr_], pr, pl)
    t0 = wl.device.lead["t0"]
    for k in range(len(e)):
        f_l = leads.fermi(e[k], wl.mu[0], wl.kt)
        f_r = leads.fermi(e[k], wl.mu[1], wl.kt)
        cgr, cgl = _waveguide_closed_form(ny, nx, t0, complex(e[k], eta2), f_l, f_r)
        assert _rel(dgr[k], cgr) < 1e-10
        assert _rel(dgl[k], cgl) < 1e-9


def test_phonon_equilibrium_fluctuation_dissipation():
    """One chemical potential for the leads and every phonon site, eta = 0
    in the device: Sigma^< = -f (Sigma^r - Sigma^r+) for every source, so
    G^< = -f (G^r - G^r+) exactly (A+ - A = Sigma^r - Sigma^r+)."""
    dev = devices.fd2d(8, 4)
    e = np.array([0.05, 0.2])
    mu = (0.1, 0.1)
    sl_, sr_, ll_, lr_ = leads.contact_self_energies(dev, e, 1e-6, mu, 0.025)
    pr, pl = phonons.diagonal_self_energies(dev, e, gamma0=1e-2, mu=mu, seed=7, equilibrium=True)
    for k in range(len(e)):
        g, gl = definition.full_greens(dev.scipy_h(), None, e[k], 0.0, dev.contacts,
                                       [sl_[k], sr_[k]], [ll_[k], lr_[k]], pr[k], pl[k])
        f = leads.fermi(e[k], 0.1, 0.025)
        assert _rel(gl, -f * (g - g.conj().T)) < 1e-11
        # and the diagonal path of the oracle agrees with the full matrices
        dgr, dgl, _ = definition.diag_greens(dev.scipy_h(), None, e[k:k + 1], 0.0, dev.contacts,
                                             [sl_[k:k + 1], sr_[k:k + 1]], [ll_[k:k + 1], lr_[k:k + 1]],
                                             pr[k:k + 1], pl[k:k + 1])
        assert _rel(dgl[0], np.diag(gl)) < 1e-12 and _rel(dgr[0], np.diag(g)) < 1e-12


def test_scba_without_coupling_is_the_phonon_free_definition():
    wl = workloads.small_grid(6, 4, n_energies=3, emin=0.05, emax=0.25, eta=1e-3, noise=0.05, seed=2)
    e, sr, sl = _problem(wl)
    h = wl.device.scipy_h()
    out = scba.scba(h, None, e, wl.eta, wl.device.contacts, sr, sl, 0.0, 0.5, 1e-12, 10)
    ref = definition.diag_greens(h, None, e, wl.eta, wl.device.contacts, sr, sl)
    assert out[5] == 1 and out[6] == 0.0
    assert _rel(out[0], ref[0]) < 1e-14 and _rel(out[1], ref[1]) < 1e-14
    assert not np.any(out[3]) and not np.any(out[4])


def test_scba_preserves_equilibrium_and_converges_to_a_fixed_point():
    """Leads at one chemical potential, eta = 0 in the device: every iterate
    keeps Sigma^<_ph = -f (Sigma^r_ph - Sigma^r_ph*) (it is D0 times a
    G^< that obeys G^< = -f (G^r - G^r*)), so the converged diagonals obey
    both identities; and the returned self-energies reproduce themselves
    when the definition is evaluated once more with them."""
    dev = devices.fd2d(8, 4)
    e = np.array([3.8, 4.2, 4.6])        # in the first transverse band (edge near 3.5 eV)
    mu = (4.2, 4.2)
    sl_, sr_, ll_, lr_ = leads.contact_self_energies(dev, e, 1e-6, mu, 0.025)
    d0 = 0.2
    dgr, dgl, _, spr, spl, it, res = scba.scba(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_],
                                               [ll_, lr_], d0, 0.7, 1e-12, 200)
    assert res < 1e-12 and 2 < it < 200
    f = leads.fermi(e, 4.2, 0.025)[:, None]
    assert _rel(dgl, -f * (dgr - dgr.conj())) < 1e-11
    assert _rel(spl, -f * (spr - spr.conj())) < 1e-11
    # fixed point: one more evaluation at the returned self-energies
    gr2, gl2, _ = definition.diag_greens(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_],
                                         [ll_, lr_], spr, spl)
    assert _rel(d0 * gr2, spr) < 1e-10 and _rel(d0 * gl2, spl) < 1e-10
    # the scattering is not negligible at this coupling
    gr0, _, _ = definition.diag_greens(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_])
    assert _rel(gr2, gr0) > 1e-2


# ---------------------------------------------------------------------------
# terminal currents
# ---------------------------------------------------------------------------

def test_terminal_current_is_landauer_and_conserved():
    """Phonon-free, eta = 0 in the device: i_L(E) = T(E) (f_L - f_R) with
    T = Tr[Gamma_L G_LR Gamma_R G_LR+] (the transmission, a different block
    of G than the contact block the current formula reads), and i_L = -i_R."""
    wl = workloads.small_grid(10, 8, n_energies=3, emin=1.2, emax=1.8, eta=0.0, mu=(1.5, 1.4), noise=0.05,
                              seed=21)
    dev = wl.device
    e = wl.energies
    sl_, sr_, ll_, lr_ = leads.contact_self_energies(dev, e, 1e-6, wl.mu, wl.kt)
    cur = definition.terminal_currents(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_])
    L, R = dev.contacts
    for k in range(len(e)):
        g, _ = definition.full_greens(dev.scipy_h(), None, e[k], 0.0, dev.contacts, [sl_[k], sr_[k]],
                                      [ll_[k], lr_[k]])
        gam_l = 1j * (sl_[k] - sl_[k].conj().T)
        gam_r = 1j * (sr_[k] - sr_[k].conj().T)
        glr = g[np.ix_(L, R)]
        t = np.trace(gam_l @ glr @ gam_r @ glr.conj().T).real
        df = leads.fermi(e[k], wl.mu[0], wl.kt) - leads.fermi(e[k], wl.mu[1], wl.kt)
        assert abs(cur[k, 0] - t * df) <= 1e-11 * abs(t * df)
        assert abs(cur[k, 0] + cur[k, 1]) <= 1e-11 * abs(cur[k, 0])
        assert t > 0.1   # energies in the first band: an open channel


def test_terminal_current_conserved_by_converged_elastic_scattering():
    """Local elastic scattering at the Born fixed point exchanges no current
    with the phonons at any energy (i D (G^<_kk G^>_kk - G^>_kk G^<_kk) = 0
    per site), so i_L + i_R = 0 still holds at eta = 0, while the current
    itself differs from the ballistic one."""
    dev = devices.fd2d(10, 8)
    e = np.array([1.3, 1.5, 1.7])
    mu = (1.5, 1.4)
    sl_, sr_, ll_, lr_ = leads.contact_self_energies(dev, e, 1e-6, mu, 0.025)
    *_, spr, spl, it, res = scba.scba(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_],
                                      0.2, 0.7, 1e-13, 300)
    assert res < 1e-13
    cur = definition.terminal_currents(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_],
                                       spr, spl)
    bal = definition.terminal_currents(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_])
    assert np.all(np.abs(cur[:, 0] + cur[:, 1]) <= 1e-9 * np.abs(cur[:, 0]))
    assert np.max(np.abs(cur[:, 0] - bal[:, 0]) / np.abs(bal[:, 0])) > 1e-2
    # a fixed, non-self-consistent phonon self-energy does exchange current
    pr, pl = phonons.diagonal_self_energies(dev, e, gamma0=2e-2, mu=(1.6, 1.3), seed=4)
    cur2 = definition.terminal_currents(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_],
                                        pr, pl)
    assert np.max(np.abs(cur2[:, 0] + cur2[:, 1]) / np.abs(cur2[:, 0])) > 1e-3


# ---------------------------------------------------------------------------
# Schroedinger-Poisson Newton step
# ---------------------------------------------------------------------------

def _sp_problem(mu=(2.2, 2.2)):
    """8 x 6 grid (first transverse band from 1.8 eV), 31 energies over the
    occupied band, eta = 0 in the device; K = 0.05 (graph Laplacian + 0.5 I),
    beta = 1, background density 1.3 n(0)."""
    dev = devices.fd2d(8, 6)
    e = np.linspace(1.7, 2.6, 31)
    w = np.full(e.size, e[1] - e[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    cE = w / (2 * np.pi)
    sl_, sr_, ll_, lr_ = leads.contact_self_energies(dev, e, 1e-7, mu, 0.025)
    h = dev.scipy_h()
    a = (h != 0).astype(float).toarray()
    np.fill_diagonal(a, 0.0)
    K = 0.05 * (np.diag(a.sum(1)) - a + 0.5 * np.eye(dev.n))
    args = (h, None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_], cE)
    n0 = gradient.density(*args)
    return dev, args, K, 1.0, 1.3 * n0


def test_density_response_symmetric_only_in_equilibrium():
    """chi = dn/dV is the Hessian of the grand potential in equilibrium
    (symmetric; exactly so at eta = 0), and not symmetric under bias."""
    dev, args, *_ = _sp_problem()
    h, _, e, eta, contacts, sr, sl, cE = args
    chi = poisson.response(h, np.zeros(dev.n), e, eta, contacts, sr, sl, cE)
    for k in (0, 17, 40):       # rows are the density's vector-Jacobian products
        e_k = np.zeros(dev.n)
        e_k[k] = 1.0
        row = gradient.density_vjp(h, np.zeros(dev.n), e, eta, contacts, sr, sl, cE, e_k)
        assert np.max(np.abs(chi[k] - row)) <= 1e-12 * np.abs(chi).max()
    assert np.abs(chi - chi.T).max() <= 1e-10 * np.abs(chi).max()
    assert np.all(np.diag(chi) < 0)          # raising V on a site lowers its density
    dev_b, args_b, *_ = _sp_problem(mu=(2.3, 2.1))
    hb, _, eb, etab, cb, srb, slb, cEb = args_b
    chib = poisson.response(hb, np.zeros(dev_b.n), eb, etab, cb, srb, slb, cEb)
    assert np.abs(chib - chib.T).max() > 1e-2 * np.abs(chib).max()


def test_newton_jacobian_matches_finite_differences_of_the_residual():
    dev, args, K, beta, nd = _sp_problem()
    h, _, e, eta, contacts, sr, sl, cE = args
    rng = np.random.default_rng(3)
    v = rng.uniform(-0.05, 0.05, dev.n)
    dv = rng.standard_normal(dev.n)
    J = K - beta * poisson.response(h, v, e, eta, contacts, sr, sl, cE)
    step = 1e-6
    fp = poisson.residual(h, v + step * dv, e, eta, contacts, sr, sl, cE, K, beta, nd)
    fm = poisson.residual(h, v - step * dv, e, eta, contacts, sr, sl, cE, K, beta, nd)
    fd = (fp - fm) / (2 * step)
    assert np.max(np.abs(J @ dv - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_newton_converges_quadratically():
    dev, args, K, beta, nd = _sp_problem()
    h, _, e, eta, contacts, sr, sl, cE = args
    v = np.zeros(dev.n)
    norms = []
    for _ in range(6):
        d, F = poisson.newton_step(h, v, e, eta, contacts, sr, sl, cE, K, beta, nd)
        norms.append(np.linalg.norm(F))
        v = v + d
    assert norms[-1] < 1e-10 * norms[0]
    # the last contracting steps square the residual (up to a modest constant)
    k = next(i for i in range(1, 6) if norms[i] < 1e-3 * norms[0])
    assert norms[k + 1] <= 10.0 * norms[k] ** 2 / norms[0] + 1e-14 * norms[0]


# ---------------------------------------------------------------------------
# lead self-energies (inputs): two independent constructions must agree
# ---------------------------------------------------------------------------

def test_sancho_rubio_matches_closed_form_fd_lead():
    nx, t0 = 6, 9.0985
    h00 = 4 * t0 * np.eye(nx) - t0 * (np.eye(nx, k=1) + np.eye(nx, k=-1))
    h01 = -t0 * np.eye(nx)
    for e in [0.05, 3.0, 12.0]:
        z = complex(e, 1e-4)
        g_right, g_left = leads.sancho_rubio(h00, h01, z)
        s_sr = h01.T @ g_left @ h01
        s_cf = leads.fd_lead_sigma(z, nx, t0)
        assert _rel(s_sr, s_cf) < 1e-9


def test_sancho_rubio_surface_dyson_fixed_point_tube():
    h00, h01 = devices.zigzag_tube_blocks(10, -2.7)
    z = complex(0.7, 1e-3)
    gr, gl = leads.sancho_rubio(h00, h01, z)
    eye = np.eye(h00.shape[0])
    assert _rel(gr, np.linalg.inv(z * eye - h00 - h01 @ gr @ h01.T)) < 1e-10
    assert _rel(gl, np.linalg.inv(z * eye - h00 - h01.T @ gl @ h01)) < 1e-10


def test_tube_transmission_counts_bloch_bands():
    h00, h01 = devices.zigzag_tube_blocks(10, -2.7)
    ks = np.linspace(0, 2 * np.pi, 2001)
    bands = np.array([np.linalg.eigvalsh(h00 + h01 * np.exp(1j * k) + h01.T * np.exp(-1j * k))
                      for k in ks])
    dev = devices.zigzag_tube(3, 10, -2.7, disorder=0.0)
    for e in [0.2, 0.75, 1.6, 2.2]:
        # right-moving channels = half the number of crossings of E over a period
        crossings = np.sum(np.diff(np.sign(bands - e), axis=0) != 0)
        n_ch = crossings // 2
        z = complex(e, 1e-8)
        s_l, s_r = leads.tube_lead_sigmas(z, h00, h01)
        g, _ = definition.full_greens(dev.scipy_h(), None, e, 1e-8, dev.contacts, [s_l, s_r],
                                      [0 * s_l, 0 * s_r])
        g1n = g[np.ix_(dev.contacts[0], dev.contacts[1])]
        t = np.trace(leads.gamma(s_l) @ g1n @ leads.gamma(s_r) @ g1n.conj().T).real
        assert abs(t - n_ch) < 1e-4, (e, t, n_ch)


def test_armchair_ribbon_transmission_counts_bloch_bands():
    """Pristine armchair ribbon (7 dimer lines): the Caroli transmission
    equals the number of right-moving Bloch channels at E (0 in the gap of
    this semiconducting ribbon), which pins the generator's cell blocks and
    the device's honeycomb graph together."""
    h00, h01 = devices.armchair_ribbon_blocks(7, -2.7)
    ks = np.linspace(0, 2 * np.pi, 2001)
    bands = np.array([np.linalg.eigvalsh(h00 + h01 * np.exp(1j * k) + h01.T * np.exp(-1j * k))
                      for k in ks])
    gap = np.min(np.abs(bands))
    assert 0.3 < gap < 1.2            # N = 7 armchair ribbons are semiconducting
    dev = devices.armchair_ribbon(4, 7, -2.7)
    for e in [0.0, 0.9, 1.5, 2.2]:
        crossings = np.sum(np.diff(np.sign(bands - e), axis=0) != 0)
        n_ch = crossings // 2
        z = complex(e, 1e-8)
        s_l, s_r = leads.tube_lead_sigmas(z, h00, h01)
        g, _ = definition.full_greens(dev.scipy_h(), None, e, 1e-8, dev.contacts, [s_l, s_r],
                                      [0 * s_l, 0 * s_r])
        g1n = g[np.ix_(dev.contacts[0], dev.contacts[1])]
        t = np.trace(leads.gamma(s_l) @ g1n @ leads.gamma(s_r) @ g1n.conj().T).real
        assert abs(t - n_ch) < 1e-4, (e, t, n_ch)


# ---------------------------------------------------------------------------
# gradient
# ---------------------------------------------------------------------------

def test_gradient_matches_central_differences():
    wl = workloads.small_grid(6, 4, n_energies=3, emin=0.02, emax=0.3, eta=1e-3)
    dev = wl.device
    e, sr, sl = _problem(wl)
    cw = wl.quad_weights()
    v0 = np.random.default_rng(7).uniform(-0.03, 0.03, dev.n)
    nbar = np.random.default_rng(8).uniform(0.5, 1.5, dev.n)
    vbar = gradient.density_vjp(dev.scipy_h(), v0, e, wl.eta, dev.contacts, sr, sl, cw, nbar)
    h = 1e-6
    for k in [0, 5, 11, 17, 23]:
        vp, vm = v0.copy(), v0.copy()
        vp[k] += h
        vm[k] -= h
        np_ = gradient.density(dev.scipy_h(), vp, e, wl.eta, dev.contacts, sr, sl, cw)
        nm = gradient.density(dev.scipy_h(), vm, e, wl.eta, dev.contacts, sr, sl, cw)
        fd = np.dot(nbar, np_ - nm) / (2 * h)
        assert abs(fd - vbar[k]) < 1e-6 * max(1.0, np.max(np.abs(vbar)))


def test_gradient_single_site_closed_form():
    """n = 1: n = c f Gamma / |A|^2 with A = z - V - Sigma, so
    dn/dV = c f Gamma 2 Re(A) / |A|^4."""
    sig = np.array([[0.1 - 0.3j]])
    z = complex(0.4, 1e-3)
    v = np.array([0.05])
    f, c = 0.7, 0.2
    gam = -2 * sig[0, 0].imag
    sless = np.array([[1j * f * gam]])
    vbar = gradient.density_vjp(np.zeros((1, 1)), v, [z.real], z.imag, [np.array([0])],
                                [sig[None]], [sless[None]], np.array([c]), np.array([1.0]))
    a = z - v[0] - sig[0, 0]
    expect = c * f * gam * 2 * a.real / abs(a) ** 4
    assert abs(vbar[0] - expect) < 1e-12 * abs(expect)


def test_sparse_lu_rows_match_dense_definition():
    from oracle import sparse
    wl = workloads.small_grid(14, 9, n_energies=3, emin=0.02, emax=0.4, eta=1e-4, noise=0.05, seed=12)
    dev = wl.device
    e, sr, sl = _problem(wl)
    v = np.random.default_rng(2).uniform(-0.02, 0.02, dev.n)
    dgr, dgl, _ = definition.diag_greens(dev.scipy_h(), v, e, wl.eta, dev.contacts, sr, sl)
    sites = np.array([0, 5, 17, 40, 63, 100, dev.n - 1])
    gr, gl = sparse.sampled_diag(dev.scipy_h(), v, e, wl.eta, dev.contacts, sr, sl, sites)
    assert _rel(gr, dgr[:, sites]) < 1e-12
    assert _rel(gl, dgl[:, sites]) < 1e-11


# ---------------------------------------------------------------------------
# G^> in its own step, and the transmission
# ---------------------------------------------------------------------------

def test_explicit_greater_differs_from_the_identity_by_the_broadening_term():
    """G^r Sigma^> G^r+ = G^< + G^r - G^r+ + 2 i eta G^r G^r+ (the identity
    holds exactly only at eta = 0): the explicit diagonal minus the
    identity's equals 2 i eta sum_j |G_kj|^2, computed from the full G."""
    wl = workloads.small_grid(9, 5, n_energies=3, eta=2e-2, noise=0.05, seed=31)
    dev = wl.device
    e, sr, sl = _problem(wl)
    dgr, dgl, dgg = definition.diag_greens(dev.scipy_h(), None, e, wl.eta, dev.contacts, sr, sl)
    exp_g = definition.diag_greater(dev.scipy_h(), None, e, wl.eta, dev.contacts, sr, sl)
    for k in range(len(e)):
        g, _ = definition.full_greens(dev.scipy_h(), None, e[k], wl.eta, dev.contacts,
                                      [s[k] for s in sr], [s[k] for s in sl])
        gg = np.sum(np.abs(g) ** 2, axis=1)
        assert _rel(exp_g[k] - dgg[k], 2j * wl.eta * gg) < 1e-10
        assert np.max(np.abs(gg)) * wl.eta > 1e-3 * np.max(np.abs(dgg[k]))  # the term is not negligible
    # at eta = 0 in the device the two coincide
    dgr0, dgl0, dgg0 = definition.diag_greens(dev.scipy_h(), None, e, 0.0, dev.contacts, sr, sl)
    exp0 = definition.diag_greater(dev.scipy_h(), None, e, 0.0, dev.contacts, sr, sl)
    assert _rel(exp0, dgg0) < 1e-11


def test_explicit_greater_in_equilibrium():
    """One chemical potential, eta = 0 in the device: G^< = -f A and
    G^> = (1 - f) A with A = G^r - G^r+, so G^> = (f - 1) / f G^< site by
    site."""
    dev = devices.fd2d(8, 5)
    e = np.array([0.05, 0.12, 0.3])
    mu, kt = (0.1, 0.1), 0.025
    sl_, sr_, ll_, lr_ = leads.contact_self_energies(dev, e, 1e-6, mu, kt)
    _, dgl, _ = definition.diag_greens(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_])
    gg = definition.diag_greater(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_])
    f = leads.fermi(e, mu[0], kt)[:, None]
    assert _rel(gg, (f - 1) / f * dgl) < 1e-10


def test_transmission_counts_channels():
    """Unit transmission per open mode of the uniform hard-wall waveguide,
    and the number of right-moving Bloch channels of the pristine (10,0)
    tube."""
    ny, nx = 10, 6
    wl = workloads.uniform_waveguide(ny, nx, n_energies=1, eta=1e-9)
    t0 = wl.device.lead["t0"]
    _, eps = leads.transverse_modes(nx, t0)
    es = np.array([0.5, 2.0, 6.0, 15.0])
    s = np.array([leads.fd_lead_sigma(complex(x, 1e-9), nx, t0) for x in es])
    t = definition.transmission(wl.device.scipy_h(), None, es, 1e-9, wl.device.contacts, [s, s])
    for x, tx in zip(es, t):
        assert abs(tx - int(np.sum((x > eps) & (x < eps + 4 * t0)))) < 1e-6
    h00, h01 = devices.zigzag_tube_blocks(10, -2.7)
    ks = np.linspace(0, 2 * np.pi, 2001)
    bands = np.array([np.linalg.eigvalsh(h00 + h01 * np.exp(1j * k) + h01.T * np.exp(-1j * k))
                      for k in ks])
    dev = devices.zigzag_tube(3, 10, -2.7, disorder=0.0)
    es = np.array([0.2, 0.75, 1.6, 2.2])
    sig = [leads.tube_lead_sigmas(complex(x, 1e-8), h00, h01) for x in es]
    t = definition.transmission(dev.scipy_h(), None, es, 1e-8, dev.contacts,
                                [np.array([a for a, _ in sig]), np.array([b for _, b in sig])])
    for x, tx in zip(es, t):
        n_ch = np.sum(np.diff(np.sign(bands - x), axis=0) != 0) // 2
        assert abs(tx - n_ch) < 1e-4, (x, tx, n_ch)


def test_transmission_is_the_landauer_current():
    """Phonon-free, eta = 0: i_L(E) = T(E) (f_L - f_R) with the terminal
    current formula (the contact block of G^< and G^>)."""
    wl = workloads.small_grid(10, 8, n_energies=3, emin=1.2, emax=1.8, eta=0.0, mu=(1.5, 1.4),
                              noise=0.05, seed=21)
    dev = wl.device
    e = wl.energies
    sl_, sr_, ll_, lr_ = leads.contact_self_energies(dev, e, 1e-6, wl.mu, wl.kt)
    cur = definition.terminal_currents(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_], [ll_, lr_])
    t = definition.transmission(dev.scipy_h(), None, e, 0.0, dev.contacts, [sl_, sr_])
    df = leads.fermi(e, wl.mu[0], wl.kt) - leads.fermi(e, wl.mu[1], wl.kt)
    assert np.all(t > 0.1)
    assert np.max(np.abs(cur[:, 0] - t * df) / np.abs(t * df)) < 1e-11
