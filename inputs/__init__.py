"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds the *inputs* of the transport problem -- the device
Hamiltonian H (real symmetric, CSR), the site coordinates, the contact site
sets, the energy grid, the retarded contact self-energies and the lesser
self-energies -- and nothing of the nested-dissection method itself.  The
problem statement these feed is the NEGF system A G^r = I, A G^< = Sigma^< G^r+
with A = E I - H - Sigma_L - Sigma_R (Section 1, equations defineGless1 and
defineA); the layered device with dense contact blocks follows Section 2.
"""
from . import devices, leads, workloads  # noqa: F401
