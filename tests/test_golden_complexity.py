"""The host operation counter and the separator tree against the complexity
tables of Section 2 (Tables 1 and 2, fixture tests/golden/complexity_tables.json):
the nested-dissection counts for diag G^r on rectangular devices stay below
the HSC coefficient (and far below RGF's), those for diag G^< on square
devices below FIND's and RGF's.  Counts follow
Section 4.1's convention (i j k per product, i^3 per inversion)."""
import json
import os

import numpy as np
import pytest

import paper_1305_1070_amd as ndg
from inputs import devices

HERE = os.path.dirname(os.path.abspath(__file__))


def _tables():
    with open(os.path.join(HERE, "golden", "complexity_tables.json")) as f:
        return json.load(f)


def _gr_ops(info):
    return (info["ops_fold_inv"] + info["ops_fold_psi"] + info["ops_fold_update"] +
            info["ops_gr_off"] + info["ops_gr_diag"])


@pytest.mark.parametrize("ny,nx", [(1024, 64), (2048, 32), (512, 128)])
def test_gr_count_below_hsc_bound_rectangular(ny, nx):
    t = _tables()["gr_rectangular_Nx_lt_Ny"]
    dev = devices.fd2d(ny, nx)
    info = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, dev.contacts, dev.coords,
                       leaf_max=16).info()
    scale2 = float(nx) * nx * ny
    assert _gr_ops(info) <= t["HSC_coeff_of_Nx2_Ny"] * scale2
    # below the RGF entry of the table by a factor that grows with Nx
    assert _gr_ops(info) < t["RGF_coeff_of_Nx3_Ny"] * float(nx) ** 3 * ny * (16.0 / nx)


@pytest.mark.parametrize("n", [64, 96, 128])
def test_gless_count_below_find_bound_square(n):
    t = _tables()["gless_square_Nx_eq_Ny"]
    dev = devices.fd2d(n, n)
    # contacts neglected, as in Section 4.1's count
    info = ndg.analyze(dev.n, dev.rowptr, dev.col, dev.val, [], dev.coords, leaf_max=16).info()
    gl = info["ops_gl_off"] + info["ops_gl_diag"]
    assert gl <= t["FIND_coeff_of_Nx3"] * float(n) ** 3
    assert gl < t["RGF_coeff_of_Nx4"] * float(n) ** 4
