"""The C ABI: every function declared in include/bura.h is exported (CPU only, no compute)."""

import os
import re

import pytest

from conftest import ROOT


def _declared():
    src = open(os.path.join(ROOT, "include", "bura.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"\b(bura_[a-z_]+)\s*\(", src))


def test_header_declares_boundary():
    names = _declared()
    for n in ("bura_plan_create", "bura_solve", "bura_submit", "bura_poll", "bura_plan_destroy",
              "bura_coefficients", "bura_strerror", "bura_plan_coeffs"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1612_04846_amd", "libbura.so"))
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    import paper_1612_04846_amd as B
    assert B.exported_symbols() == _declared()


def test_strerror_and_defaults():
    import paper_1612_04846_amd as B
    assert B.bura_strerror(B.BURA_OK) == "ok"
    assert "invalid" in B.bura_strerror(B.BURA_EINVAL)
    o = B.bura_opts_default()
    assert o.tol == 1e-12 and o.precision == B.BURA_MIXED and o.nu_pre == 2 and o.nrhs_max == 1


@pytest.mark.parametrize("alpha,k,beta,code", [(0.0, 5, 1, -1), (1.0, 5, 1, -1), (0.5, 0, 1, -1),
                                               (0.5, 17, 1, -1), (0.5, 5, 3, -2)])
def test_coefficients_argument_errors(alpha, k, beta, code):
    import paper_1612_04846_amd as B
    with pytest.raises(B.BuraError) as ei:
        B.bura_coefficients(alpha, k, beta)
    assert ei.value.code == code
