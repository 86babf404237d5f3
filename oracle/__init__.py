"""CPU oracle for the nested-dissection NEGF hot path -- TEST INFRASTRUCTURE.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import, call or execute anything in this package.  The product path (the HIP
library and its Python binding) never touches it, and this package never
imports the product: the two share no code.  The only shared module is the
seeded input generator package `inputs`, which holds none of the method's
arithmetic.

What it computes (all complex128 / float64):
  * definition.py -- the problem statement itself (Section 1, equations
    defineGless1 and defineA): A = zI - H - diag(V) - Sigma_L - Sigma_R
    - diag(Sigma_Phonon) (the phonon term optional and diagonal, its lesser
    part added to Sigma^<), G^r = A^{-1} by dense LU, G^< = G^r Sigma^< G^r+, and
    G^> := G^< + G^r - G^r+ on the diagonal.  The nested-dissection method is
    exact (Sections 1 and 3: every stored entry of G^(0) and P^(0) equals the
    corresponding entry of G^r and G^<), so this definition is the oracle.
  * rgf.py -- the layer-by-layer recursive Green's function method reviewed
    in Section 2 (fold left-to-right, extract right-to-left), for devices too
    large for dense inversion.
  * brute.py -- the definition again in 50-digit arithmetic (mpmath), no
    LAPACK, for tiny grids.
  * gradient.py -- d(density)/d(on-site potential) from the dense definition.
  * scba.py -- the self-consistent Born loop of local elastic phonon
    scattering (Sigma_ph = d0 diag G) over the dense definition.
  * poisson.py -- the Newton step of the Schroedinger-Poisson problem,
    F = K V - beta (n(V) - n_D), with dn/dV assembled from gradient.py.
  * definition.terminal_currents -- the current spectral density per contact,
    Tr[Sigma^< G^> - Sigma^> G^<] over the contact block.

Pins (tests/test_oracle_*.py, marked "not gpu"): mpmath brute force, the
closed-form Green's function of the uniform hard-wall waveguide (retarded
and lesser, exact at complex energy), unit transmission per open mode, the
anti-Hermiticity of G^<, the identity G^r - G^r+ = -i G^r Gamma G^r+ with
Gamma including the 2 eta broadening, equilibrium G^< = -f (G^r - G^r+) up to
the eta term, the paper's printed 3-cluster and 3-level block formulas, and
central finite differences for the gradient.  With phonons: the 50-digit brute
force, the waveguide closed form at z = E + i(eta + gamma/2) for a uniform
Sigma^r_ph = -i gamma/2, and the fluctuation-dissipation identity
G^< = -f (G^r - G^r+) at eta = 0 in equilibrium.  Born loop: D0 = 0, the
fluctuation-dissipation pairs of every iterate, the fixed point.  Currents:
Landauer's Tr[Gamma_L G_LR Gamma_R G_LR+] (f_L - f_R) and conservation.
Newton step: dn/dV symmetric in equilibrium, central differences of F,
quadratic convergence.
"""
