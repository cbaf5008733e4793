"""One context used from several host threads at once (the C calls release
the interpreter lock, so they really overlap): every entry point must give
the result it gives alone, while the serving worker runs beside them.
A context serialises its device work, so the comparison is bit for bit on
the double-double value."""
import sys
import threading

import numpy as np
import pytest

from paper_2109_04528_amd import inputs as gen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_threads_share_one_context():
    from paper_2109_04528_amd import Context
    mats = [gen.random_O(n, 900 + n, 0.4, 1.1, 0.8) for n in (9, 14, 17, 20, 12)]
    state = gen.random_O(14, 950, 0.5, 1.0, 0.7)
    pats = [0b11, 0b1010101, 0b11110000111, (1 << 14) - 1]
    say("case four threads on one context")
    with Context(device=0) as ctx:
        want = [ctx.eval(O) for O in mats]
        want_batch = ctx.eval_batch(mats)
        want_click, _ = ctx.click_probs(state, pats)
        errors = []

        def worker(tid):
            try:
                for it in range(6):
                    j = (tid + it) % len(mats)
                    r = ctx.eval(mats[j])
                    assert (r.tor, r.tor_lo) == (want[j].tor, want[j].tor_lo)
                    if it % 2 == 0:
                        rb = ctx.eval_batch(mats)
                        assert all((x.tor, x.tor_lo) == (y.tor, y.tor_lo) for x, y in zip(rb, want_batch))
                    else:
                        p, _ = ctx.click_probs(state, pats)
                        assert np.array_equal(p, want_click)
                    t = ctx.submit(mats[j])
                    ctx.drain(60000)
                    s = ctx.poll(t)
                    assert s is not None and (s.tor, s.tor_lo) == (want[j].tor, want[j].tor_lo)
            except Exception as e:  # reported by the main thread
                errors.append((tid, repr(e)))

        ths = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
        for th in ths:
            th.start()
        for th in ths:
            th.join(120)
        assert not any(th.is_alive() for th in ths)
        say(f"  errors: {errors}")
        assert not errors
