"""tor_eval_static, the entry point for callers that cannot allocate: the
same value as tor_eval through the C ABI, on two calls in a row (the
second with a smaller matrix, so the array still holds the first call's
data), from host and from device memory, and the scratch-size limit."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2109_04528_amd import inputs as gen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same_value(a, b):
    # the double-double sum is exact, so the value is the same bit for bit
    return (a.tor, a.tor_lo, a.path, a.status) == (b.tor, b.tor_lo, b.path, b.status)


def test_static_equals_eval_two_calls_host_input():
    from paper_2109_04528_amd import Context
    big = gen.random_O(30, 0, 0.3, 1.2, 0.9)
    small = gen.random_O(17, 3, 0.5, 1.0, 0.7)
    with Context(device=0) as ctx:
        for O in (big, small):
            n = O.shape[0] // 2
            say(f"case static entry point, host input n={n}")
            a = ctx.eval_static(O)
            b = ctx.eval(O)
            say(f"  static={a.value!r} eval={b.value!r} path={a.path} ms={a.device_ms:.3f}/{b.device_ms:.3f}")
            assert same_value(a, b)
            assert abs(a.sum_abs - b.sum_abs) <= 1e-12 * b.sum_abs
            assert a.subsets == b.subsets == 1 << n


def test_static_equals_eval_device_input_and_complex_path():
    import torch
    from paper_2109_04528_amd import Context, TOR_FORCE_COMPLEX, TOR_INPUT_DEVICE
    mats = [gen.random_O(24, 1, 0.5, 1.0, 0.7), gen.random_hpd_O(12, 5, 0.05, 0.9)]
    with Context(device=0, flags=TOR_INPUT_DEVICE) as ctx:
        for O in mats:
            t = torch.from_numpy(O).to("cuda:0")
            say(f"case static entry point, device input n={O.shape[0] // 2}")
            assert same_value(ctx.eval_static(t), ctx.eval(t))
    with Context(device=0, flags=TOR_FORCE_COMPLEX) as ctx:
        for O in (gen.random_O(22, 2, 0.3, 1.2, 0.9), gen.random_O(9, 4, 0.3, 1.2, 0.9)):
            say(f"case static entry point, complex path n={O.shape[0] // 2}")
            a, b = ctx.eval_static(O), ctx.eval(O)
            assert a.path == 2 and same_value(a, b)


def test_static_limits_and_errors():
    from paper_2109_04528_amd import Context, TorError, TOR_E_INVAL, TOR_E_NOT_PD, TOR_E_SCRATCH, TOR_FORCE_COMPLEX
    from paper_2109_04528_amd import _lib
    say("case static entry point: limits and errors")
    with Context(device=0, flags=TOR_FORCE_COMPLEX) as ctx:
        # the complex path's stacks at n = 32 exceed the array
        with pytest.raises(TorError) as ei:
            ctx.eval_static(gen.random_O(32, 0, 0.5, 1.0, 0.7))
        assert ei.value.code == TOR_E_SCRATCH
        # the array still serves the next call
        O = gen.random_O(14, 6, 0.5, 1.0, 0.7)
        assert same_value(ctx.eval_static(O), ctx.eval(O))
    with Context(device=0) as ctx:
        with pytest.raises(TorError) as ei:
            ctx.eval_static(gen.random_O(6, 1) + 2.0 * np.eye(12))
        assert ei.value.code == TOR_E_NOT_PD
        bad = gen.random_O(6, 1)
        bad[3, 1] = np.nan
        with pytest.raises(TorError) as ei:
            ctx.eval_static(bad)
        assert ei.value.code == TOR_E_INVAL
        r = _lib.tor_result()
        assert _lib.load().tor_eval_static(None, 1, None, 2, ctypes.byref(r)) == TOR_E_INVAL
        assert ctx.eval_static(gen.vacuum_O(0)).value == 1.0
