"""The C oracle built with the host AddressSanitizer and UndefinedBehavior-
Sanitizer (gcc; every diagnostic fatal) runs, in a child process, a small DM
field, its transpose, the tensor at single offsets, the Newell f and g, the
SP kernel, potential and field: no out-of-bounds access, use after free or
undefined behaviour, and the same values as the regular build."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SHAPE, CELL, MS = (5, 4, 3), (2e-9, 1.5e-9, 3e-9), 8e5

CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[3])
import oracle
lib = oracle.load(sys.argv[1])
shape, cell, Ms = (5, 4, 3), (2e-9, 1.5e-9, 3e-9), 8e5
rng = np.random.default_rng(5)
m = rng.standard_normal((3,) + shape[::-1])
o = oracle.Oracle(shape, cell, lib=lib)
H = o.field(m, Ms)
HT = o.field_T(m, Ms)
s = oracle.SPOracle(shape, cell, lib=lib)
Hs = s.field(m, Ms)
fg = np.array([lib.oracle_f(1.3, -0.7, 2.1), lib.oracle_g(0.4, 1.9, -1.2),
               lib.oracle_tensor_at(3, 2, -1, 1, *cell)])
np.savez(sys.argv[2], N=o.Noct, H=H, HT=HT, S=s.Soct, Hs=Hs, fg=fg)
"""


def _reference(lib):
    rng = np.random.default_rng(5)
    m = rng.standard_normal((3,) + SHAPE[::-1])
    o = oracle.Oracle(SHAPE, CELL, lib=lib)
    s = oracle.SPOracle(SHAPE, CELL, lib=lib)
    fg = np.array([lib.oracle_f(1.3, -0.7, 2.1), lib.oracle_g(0.4, 1.9, -1.2),
                   lib.oracle_tensor_at(3, 2, -1, 1, *CELL)])
    return dict(N=o.Noct, H=o.field(m, MS), HT=o.field_T(m, MS), S=s.Soct, Hs=s.field(m, MS), fg=fg)


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isfile(os.path.realpath(asan)):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib_path = str(tmp_path / "oracle_sanitized.so")
    oracle.build(force=True, out=lib_path,
                 extra_flags=["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                              "-fno-omit-frame-pointer", "-g"])
    out = str(tmp_path / "values.npz")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", CHILD, lib_path, out, ROOT], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    got = np.load(out)
    ref = _reference(oracle.load())
    for k, v in ref.items():
        # the same arithmetic; the sanitized build may contract or order differently
        assert np.allclose(got[k], v, rtol=1e-13, atol=1e-13 * np.abs(v).max()), k
