"""The C ABI library loads and exports every symbol include/nk.h declares.

CPU-only: no compute call is made.  Argument checks that fail before any
device work are exercised too.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nk.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nk_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("nk_lattice_create", "nk_gauge_set", "nk_apply_dw", "nk_sign_apply", "nk_sign_apply_device",
              "nk_small_sign", "nk_rh_sign", "nk_krylov_basis_device", "nk_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_0910_2918_amd import nk

    lib = nk.library()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(nk.EXPORTS)


def test_version_and_defaults():
    from paper_0910_2918_amd import nk

    assert "gfx950" in nk.nk_version()
    p = nk.nk_sign_params_default()
    assert p.m_w == -1.0 and p.k == 100 and p.ell == 0 and p.nrhs == 1
    assert p.rh_tol == 1e-13 and p.rh_maxit == 100 and p.check_every == 50


@pytest.mark.parametrize("dims", [(4, 4, 4, 3), (0, 4, 4, 4), (4, 4, 1, 4)])
def test_bad_dims_rejected(dims):
    from paper_0910_2918_amd import nk

    with pytest.raises(nk.NKError) as ei:
        nk.nk_lattice_create(dims)
    assert ei.value.code == nk.NK_EINVAL
    assert "even" in nk.nk_last_error()


def test_rh_sign_rejects_bad_sizes():
    import numpy as np

    from paper_0910_2918_amd import nk

    s = np.zeros((1, 4, 4), np.complex128)
    with pytest.raises(nk.NKError):
        nk.nk_rh_sign(s, n=[5])


def test_rh_tile_force_and_choice_arguments():
    """Host-side checks of the blocked inverse's shape control (no device work)."""
    from paper_0910_2918_amd import nk

    with pytest.raises(nk.NKError) as ei:
        nk.nk_rh_tile_force(3, 512, 64)  # no shape with 3 rows per thread
    assert ei.value.code == nk.NK_EINVAL
    with pytest.raises(nk.NKError):
        nk.nk_rh_tile_force(1, 512, 48)  # no 48 tile
    nk.nk_rh_tile_force(2, 512, 32)
    nk.nk_rh_tile_force(0, 0, 0)
    assert nk.nk_rh_tile_choice(300, 1) is None  # nothing tuned in this process
    with pytest.raises(nk.NKError):
        nk.nk_rh_tile_choice(0, 1)


def test_small_sign_rejects_ell_above_k():
    import numpy as np

    from paper_0910_2918_amd import nk

    a = np.ones(4, np.complex128)
    with pytest.raises(nk.NKError):
        nk.nk_small_sign(4, 5, True, a, a, a)


def test_struct_layout_matches_header(tmp_path):
    """ctypes mirrors of the structs agree with the C compiler's layout."""
    import shutil
    import subprocess

    from paper_0910_2918_amd import nk

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    fields = {"nk_sign_params": [f for f, _ in nk.nk_sign_params._fields_],
              "nk_sign_info": [f for f, _ in nk.nk_sign_info._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "nk.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for st, fs in fields.items():
        cls = getattr(nk, st)
        assert int(out[st]) == __import__("ctypes").sizeof(cls)
        for f in fs:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)
