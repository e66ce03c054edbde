"""Host-side checks of the C-ABI library (no GPU needed).

* the shared library loads and exports every function include/pbt.h declares;
* its own quadrature tables (written independently of the oracle's) are
  exact on monomials up to their degree, and agree with the oracle's;
* parameter validation rejects out-of-range values before touching a device.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_1506_03745_amd as P
from paper_1506_03745_amd import pbt as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "pbt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pbt_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_header_function():
    L = P.lib()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTS)


DEGREE = {1: 1, 3: 2, 4: 3, 7: 5, 19: 9}


@pytest.mark.parametrize("npts", sorted(DEGREE))
def test_library_triangle_rules_exact(npts):
    bary, w = P.quadrature_rule(npts)
    assert abs(w.sum() - 1) < 1e-14
    for d in range(DEGREE[npts] + 1):
        for a in range(d + 1):
            for b in range(d - a + 1):
                c = d - a - b
                exact = 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(d + 2)
                q = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c)
                assert abs(q - exact) < 1e-13


@pytest.mark.parametrize("npts", sorted(DEGREE))
def test_library_rules_match_oracle_as_sets(npts):
    from oracle.quadrature import triangle_rule
    b1, w1 = P.quadrature_rule(npts)
    b2, w2 = triangle_rule(npts)
    k1 = sorted(zip(np.round(b1, 12).tolist(), np.round(w1, 12).tolist()))
    k2 = sorted(zip(np.round(b2, 12).tolist(), np.round(w2, 12).tolist()))
    assert k1 == k2


@pytest.mark.parametrize("n", [1, 2, 5, 9, 16])
def test_library_gauss_legendre(n):
    t, w = P.quadrature_rule(-n)
    for k in range(2 * n):
        assert abs(np.sum(w * t ** k) - 1.0 / (k + 1)) < 1e-14
    assert np.all(np.diff(np.sort(t)) > 0) and np.all((t > 0) & (t < 1))


def test_invalid_rule_and_params_rejected_on_host():
    with pytest.raises(B.PbtError):
        P.quadrature_rule(5)
    for bad in (dict(theta=1.5), dict(theta=0.0), dict(taylor_p=12), dict(k_far=2), dict(k_near=6),
                dict(ncrit=0), dict(tol=0.0), dict(restart=0), dict(restart=1025), dict(taylor_p=9),
                dict(near_factor=0.0), dict(near_factor=-1.0), dict(near_factor=float("nan")), dict(precond=2)):
        p = B.default_params()
        for k, v in bad.items():
            setattr(p, k, v)
        h = ctypes.c_void_p()
        assert P.lib().pbt_create(ctypes.byref(h), 0, ctypes.byref(p)) == 1, bad


def test_struct_layouts_match_header():
    # field order and sizes of the two public structs
    assert ctypes.sizeof(B.PbtParams) == 5 * 4 + 4 + 8 + 8 + 4 * 4 + 8 + 8
    assert ctypes.sizeof(B.PbtResult) == 4 * 8 + 2 * 4 + 3 * 8 + 4 * 8 + 2 * 4 + 8


def test_richardson_helpers_recover_order_and_limit():
    from paper_1506_03745_amd.convergence import observed_order, richardson
    # f = a + b N^-p on meshes with N, 4N, 16N panels
    a, b, p = 0.0614, 0.37, 1.0
    f = [a + b * (0.25 ** k) ** p for k in range(3)]
    assert abs(observed_order(*f) - p) < 1e-12
    assert abs(richardson(f[1], f[2], observed_order(*f)) - a) < 1e-12
    g = [a + b * (0.25 ** k) ** 2 for k in range(3)]
    assert abs(observed_order(*g) - 2.0) < 1e-12
