"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol include/lq.h declares, and its host-only routines validate arguments."""
import os
import re

import numpy as np
import pytest

from paper_2201_09004_amd import lq as L
from oracle import overlap as OV

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lq.h")).read()
    return sorted(set(re.findall(r"^(?:lq_status|const char \*)\s*(lq_[a-z0-9_]+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not L.lib_available():
        pytest.fail("liblq.so is not built (run __graft_entry__.build())")
    return L.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(L.EXPORTS)


def test_version_and_error_string(lib):
    assert "gfx950" in L.lq_version()
    assert isinstance(L.last_error(), str)


def test_cheb_coeffs_match_oracle(lib):
    """Host routine of the library vs the oracle's interpolation coefficients."""
    for a, b, N in [(0.3, 40.0, 10), (0.29, 48.0, 200), (1e-3, 1.0, 57)]:
        c_lib = L.lq_cheb_coeffs(a, b, N)
        c_or = OV.cheb_coeffs(a, b, N)
        assert np.abs(c_lib - c_or).max() < 1e-13 * max(1.0, np.abs(c_or).max())


@pytest.mark.parametrize("args", [(0.0, 1.0, 4), (2.0, 1.0, 4), (0.5, 1.0, -1)])
def test_cheb_coeffs_rejects_bad_interval(lib, args):
    with pytest.raises(L.LqError) as e:
        L.lq_cheb_coeffs(*args)
    assert e.value.code == L.LQ_EINVAL


def test_struct_layouts_match_header(lib):
    import ctypes as C
    # sizes follow the natural C layout of the structs in include/lq.h
    assert C.sizeof(L.lq_geom) == 20
    assert C.sizeof(L.lq_action) == 80
    assert C.sizeof(L.lq_stats) == 48
    assert C.sizeof(L.lq_mg_params) == 80


def test_struct_layouts_match_the_c_compiler(lib, tmp_path):
    """Every field offset and struct size of the binding equals what gcc makes
    of include/lq.h."""
    import ctypes as C
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = [L.lq_geom, L.lq_action, L.lq_params, L.lq_stats, L.lq_mg_params]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lq.h"', "int main(void) {"]
    for S in structs:
        n = S.__name__
        lines.append(f'printf("{n} %zu\\n", sizeof({n}));')
        for f, _ in S._fields_:
            lines.append(f'printf("{n}.{f} %zu\\n", offsetof({n}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for S in structs:
        n = S.__name__
        assert int(got[n]) == C.sizeof(S), n
        for f, _ in S._fields_:
            assert int(got[f"{n}.{f}"]) == getattr(S, f).offset, (n, f)


def test_init_without_device_is_an_error_not_a_crash(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(L.LqError) as e:
        L.lq_init(0)
    assert e.value.code == L.LQ_EDEVICE
