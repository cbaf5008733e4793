"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only): a driver runs every precision mode, a threaded
subtree restriction and one subset's determinant on a seeded input, with
any sanitizer report fatal, and must print exactly what the regular build
computes."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2109_04528_amd import inputs as gen

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan():
    n = 7
    O = np.ascontiguousarray(gen.random_O(n, 12, 0.3, 1.2, 0.9))
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitized")
        flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
        subprocess.run(["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-pthread"] + flags +
                       [os.path.join(ROOT, "oracle", "tor_oracle.c"), os.path.join(HERE, "oracle_sanitize_main.c"),
                        "-o", exe, "-lquadmath", "-lm"], check=True)
        path = os.path.join(tmp, "O.bin")
        O.tofile(path)
        # the environment is passed on as it is; a library preloaded ahead of
        # the sanitizer runtime is allowed rather than removed
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        res = subprocess.run([exe, path, str(n)], capture_output=True, text=True, env=env, timeout=120)
        assert res.returncode == 0, res.stderr[-3000:]
        assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-3000:]
        got = [float(v) for v in res.stdout.split()]
    want = []
    for mode in (orc.F64, orc.LD, orc.QUAD):
        r = orc.tor(O, mode=mode)
        want += [r.value, r.sum_abs]
    want.append(orc.tor(O, mode=orc.F64, fix_mask=3, fix_val=1).value)
    want += list(orc.det(O, (1 << n) - 2))
    assert len(got) == len(want)
    # the same source and flags that fix rounding (no contraction): the same
    # numbers, to the last bit for the FP64 and extended sums
    for g, w in zip(got, want):
        assert g == w or abs(g - w) <= 4e-16 * abs(w), (g, w)
