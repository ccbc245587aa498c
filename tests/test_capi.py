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


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structures have the C header's sizes and field offsets
    (a C program built here with gcc prints them)."""
    import ctypes
    import subprocess
    import paper_1612_04846_amd as B
    structs = {"bura_grid_t": B.bura_grid_t, "bura_opts_t": B.bura_opts_t, "bura_report_t": B.bura_report_t,
               "bura_request_t": B.bura_request_t, "bura_server_stats_t": B.bura_server_stats_t}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bura.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_tile_variant_count_matches_header():
    import paper_1612_04846_amd as B
    src = open(os.path.join(ROOT, "include", "bura.h")).read()
    m = re.search(r"#define BURA_TILE_VARIANTS (\d+)", src)
    assert m and int(m.group(1)) == B.BURA_TILE_VARIANTS


def test_slot_argument_marshalling():
    """Per-rhs terms are laid out row by row, max_terms apart (no GPU needed)."""
    import paper_1612_04846_amd as B
    nt, w, s, t = B._slot_arrays(4, [([1.0, 2.0], [0.0, 0.5]), ([3.0], [1.5])], [1e-10, 1e-12])
    assert list(nt) == [2, 1]
    assert list(w) == [1.0, 2.0, 0.0, 0.0, 3.0, 0.0, 0.0, 0.0]
    assert list(s) == [0.0, 0.5, 0.0, 0.0, 1.5, 0.0, 0.0, 0.0]
    assert list(t) == [1e-10, 1e-12]
    assert B._slot_arrays(2, [([1.0], [0.0])], None)[3] is None
    with pytest.raises(ValueError):
        B._slot_arrays(2, [([1.0, 2.0, 3.0], [0.0, 0.0, 0.0])], None)
    with pytest.raises(ValueError):
        B._slot_arrays(2, [([1.0, 2.0], [0.0])], None)


@pytest.mark.parametrize("field,value", [("nu_post", 3), ("nu_pre", 4), ("check_every", 0)])
def test_plan_rejects_asymmetric_or_unsupported_smoothing(field, value):
    """A V-cycle with nu_pre != nu_post is not symmetric (PCG needs an SPD
    preconditioner) and the sweep weights cover 1..3 sweeps: BURA_EINVAL, on
    the host, before any device work."""
    import paper_1612_04846_amd as B
    o = B.bura_opts_default(precision=B.BURA_FP64)
    setattr(o, field, value)
    if field == "nu_pre":
        o.nu_post = value
    with pytest.raises(B.BuraError) as ei:
        B.bura_plan_create(2, 31, 0.5, 5, o)
    assert ei.value.code == B.BURA_EINVAL


def test_unscaled_rhs_needs_a_fractional_power():
    """rhs_unscaled applies Lambda^-alpha: caller-given terms carry no alpha, so
    the rational plans refuse it, as does a value other than 0 or 1."""
    import paper_1612_04846_amd as B
    o = B.bura_opts_default(precision=B.BURA_FP64)
    g, _ = B._grid(2, 31, None, 0.0, 1)
    w = (B.ctypes.c_double * 1)(1.0)
    sh = (B.ctypes.c_double * 1)(0.0)
    h = B._P()
    assert B._lib.bura_plan_create_rational(B.ctypes.byref(g), 1, w, sh, B.ctypes.byref(o), B.ctypes.byref(h)) \
        == B.BURA_EINVAL
    g2, _ = B._grid(2, 31, None, 0.0, 2)
    assert B._lib.bura_plan_create(B.ctypes.byref(g2), 0.5, 1, 5, B.ctypes.byref(o), B.ctypes.byref(h)) \
        == B.BURA_EINVAL


def test_unknown_tickets_and_null_arguments():
    import paper_1612_04846_amd as B
    assert B.bura_poll(987654321)[0] == B.BURA_EINVAL
    assert B.bura_wait(987654321)[0] == B.BURA_EINVAL
    t = B.ctypes.c_uint64(5)
    assert B._lib.bura_submit(None, None, None, 1, 0.0, B.ctypes.byref(t)) == B.BURA_EINVAL
    assert t.value == 0


def test_sinc_kprime_inverts_the_system_count():
    """Section 5.3: k_Q = pi^2/(4 alpha (1-alpha) k'^2)."""
    import math
    import paper_1612_04846_amd as B
    for alpha, kq in ((0.25, 9), (0.5, 7), (0.75, 6), (0.5, 19)):
        kp = B.sinc_kprime(alpha, kq)
        assert abs(math.pi ** 2 / (4 * alpha * (1 - alpha) * kp * kp) - kq) <= 1e-12 * kq
    with pytest.raises(B.BuraError):
        B.sinc_kprime(1.0, 9)
    with pytest.raises(B.BuraError):
        B.sinc_kprime(0.5, 0.0)


def test_err_tol_needs_mixed_precision_and_no_stages():
    """The certified-bound enforcement refines FP64 iterates of the mixed
    refinement loop, and sequential forms have no per-output bound."""
    import paper_1612_04846_amd as B
    with pytest.raises(B.BuraError) as ei:
        B.bura_plan_create(2, 31, 0.5, 5, B.bura_opts_default(precision=B.BURA_FP64, err_tol=1e-8))
    assert ei.value.code == B.BURA_EUNSUPPORTED
    with pytest.raises(B.BuraError) as ei:
        B.bura_plan_create_multistep(2, 31, [0.5, 0.25], [5, 5], B.bura_opts_default(err_tol=1e-8))
    assert ei.value.code == B.BURA_EUNSUPPORTED
    with pytest.raises(B.BuraError) as ei:
        B.bura_plan_create(2, 31, 0.5, 5, B.bura_opts_default(err_tol=-1.0))
    assert ei.value.code == B.BURA_EINVAL


def test_unknown_variant_bits_are_rejected():
    """opts.variant takes only the documented alternative code paths."""
    import paper_1612_04846_amd as B
    allbits = (B.BURA_VARIANT_UNFUSED | B.BURA_VARIANT_NO_FOLDXR | B.BURA_VARIANT_FOLD_SCALARS
               | B.BURA_VARIANT_NO_GRAPH)
    assert B.bura_opts_default().variant == 0
    for v in (16, allbits | 32, -1):
        with pytest.raises(B.BuraError) as ei:
            B.bura_plan_create(2, 31, 0.5, 5, B.bura_opts_default(variant=v))
        assert ei.value.code == B.BURA_EINVAL
