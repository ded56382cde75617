"""The C-ABI library loads and exports what include/gpe.h declares (CPU only:
no call here touches a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "gpe.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(gpe_\w+)\s*\(", txt, re.M)))


def _lib():
    from paper_1504_02891_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("libgpe.so not built")
    return _native


def test_every_declared_symbol_is_exported():
    nat = _lib()
    L = ctypes.CDLL(nat.LIB_PATH)
    decl = _declared()
    assert len(decl) >= 12
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(nat.EXPORTS)


def test_struct_layouts_match_the_header(tmp_path):
    # every field of the ctypes mirrors sits at the header's offset (a
    # misplaced field would silently set a different C option)
    nat = _lib()
    structs = (("gpe_problem", nat.Problem), ("gpe_options", nat.Options), ("gpe_result", nat.Result))
    lines = []
    for cname, py in structs:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gpe.h"\n'
                   'int main(void){' + "".join(lines) + 'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = []
    for cname, py in structs:
        want.append(ctypes.sizeof(py))
        want.extend(getattr(py, fname).offset for fname, _ in py._fields_)
    assert got == want


def test_host_only_entry_points():
    nat = _lib()
    L = nat.lib()
    o = nat.Options()
    L.gpe_options_default(ctypes.byref(o))
    assert (o.precision, o.algorithm, o.k_init, o.k_sub) == (nat.GPE_PREC_FP64, nat.GPE_ALG2, 100, 200)
    assert o.tol == 1e-6 and o.rho1 == 1e-4 and o.eta == 0.85 and o.sigma == 0.5
    assert o.renorm_tol == 1e-14 and o.tau0 == 1e-3
    assert L.gpe_strerror(-1) == b"invalid argument"
    assert L.gpe_strerror(1).startswith(b"not converged")
    # null arguments are rejected before any device work
    assert L.gpe_ctx_create(None, 0, None) == nat.GPE_EINVAL
    assert L.gpe_apply_h(None, None, 0, None, None, None) == nat.GPE_EINVAL
    assert L.gpe_solve(None, None, None, None, None) == nat.GPE_EINVAL
    assert L.gpe_set_plan(None, None, 0, None, None, 0) == nat.GPE_EINVAL
    assert L.gpe_hess_vec(None, None, 0, None, None, 0.0, None) == nat.GPE_EINVAL
    assert L.gpe_retract(None, 1, 0, None, None, 0.1, None, None) == nat.GPE_EINVAL


def test_binding_argument_counts_match_the_header():
    # each ctypes prototype has as many parameters as the header declares
    nat = _lib()
    L = nat.lib()
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    decls = re.findall(r"^\s*(?:int|void|const char\*)\s+(gpe_\w+)\s*\(([^)]*)\)", txt, re.M)
    assert len(decls) == len(nat.EXPORTS)
    for name, params in decls:
        params = params.strip()
        n = 0 if params in ("", "void") else params.count(",") + 1
        assert len(getattr(L, name).argtypes) == n, name


def test_oracle_and_library_defaults_agree():
    # the oracle's constants and the library's defaults are the same readings
    nat = _lib()
    from oracle.newton import Options
    o = nat.Options()
    nat.lib().gpe_options_default(ctypes.byref(o))
    ref = Options()
    for k in ("k_init", "k_sub", "max_outer", "tau0", "rho1", "eta", "sigma", "m_max", "renorm_tol",
              "eta1", "eta2", "gamma_shrink", "gamma_grow", "delta0", "delta_min", "delta_max"):
        assert getattr(o, k) == getattr(ref, k), k
