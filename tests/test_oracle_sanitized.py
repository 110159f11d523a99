"""The oracle's C helper (oracle/sparse_ref.c) built with gcc's address and
undefined-behaviour sanitizers, run through the factorisation pins in a
subprocess (the sanitizer runtime has to be loaded first).  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHECK = r"""
import sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
from oracle import lp_oracle as O
import test_oracle_pins as T
import numpy as np
assert T.pin_incomplete_factorizations(O)
assert T.pin_red_black_factorizations(O)
from paper_2203_13675_amd import synth
rng = np.random.default_rng(16)
psi = synth.wrap_measurement(np.cumsum(rng.normal(0, 0.5, 50))[None, :])
for pc in ("ilu0", "ic0", "ssor", "ilu0_rb", "ssor_rb"):
    r = O.unwrap(psi, p=0.0, precond=pc, k_max=2, outer_tol=0.0)
    assert max(r.relres) <= 1e-6, (pc, r.relres)
psi, _ = synth.peaks_map(24, 20, scale=3.0, sigma=0.3, seed=3)
mask = np.ones((24, 20))
mask[5:9, 6:11] = 0.0
for pc in ("ilu0", "ic0", "ssor"):
    r = O.unwrap(psi, mask, p=0.0, precond=pc, k_max=2, outer_tol=0.0)
    assert max(r.relres) <= 1e-6, (pc, r.relres)
print("SANITIZED_OK")
"""


def _runtime(name):
    out = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_sparse_helper_under_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no address-sanitizer runtime here")
    so = str(tmp_path / "liblp_oracle_sparse_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fPIC", "-shared", "-o", so,
                           os.path.join(ROOT, "oracle", "sparse_ref.c"), "-lm"])
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["LP_ORACLE_SPARSE_SO"] = so
    code = CHECK.format(root=ROOT, tests=os.path.join(ROOT, "tests"))
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    assert p.returncode == 0 and "SANITIZED_OK" in p.stdout, p.stdout[-3000:] + p.stderr[-3000:]
