"""The C ABI: the library loads without a GPU, exports every function that
include/pw.h declares, and its host-side basis enumeration equals the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1907_06821_amd import synth
from oracle.basis import plane_wave_basis

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pw_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    import paper_1907_06821_amd as pw
    lib = ctypes.CDLL(str(pw.LIBPATH))
    names = _declared()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(pw.EXPORTS) == names


@pytest.mark.parametrize("cfg", [1, 2])
def test_library_basis_equals_oracle(cfg):
    import paper_1907_06821_amd as pw
    p = synth.config(cfg)
    got = pw.basis_miller(p.grid, p.cell, p.ecut)
    ref, _ = plane_wave_basis(p.cell, p.ecut)
    assert np.array_equal(got, ref)


def test_library_basis_kpoint_and_errors():
    import paper_1907_06821_amd as pw
    p = synth.small_nonlocal_problem(kpt=(0.11, -0.23, 0.07))
    got = pw.basis_miller(p.grid, p.cell, p.ecut, p.kpt)
    ref, _ = plane_wave_basis(p.cell, p.ecut, p.kpt)
    assert np.array_equal(got, ref)
    with pytest.raises(pw.PwError) as e:
        pw.basis_miller((16, 16, 16), (10.0, 10.0, -1.0), 6.0)
    assert e.value.status == pw.PW_EINVAL


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
