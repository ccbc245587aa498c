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
