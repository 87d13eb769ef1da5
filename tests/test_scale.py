"""The scale choice (host-only C-ABI call, no GPU needed) against a brute force over every
breakpoint of the paper's objective, and its limits."""
import numpy as np
import pytest

from oracle import scale
from paper_1602_08393_amd import wmh


def _lib_or_skip():
    try:
        wmh.load()
    except Exception as e:  # library not built here
        pytest.skip(f"libwmh not built: {e}")


@pytest.mark.parametrize("seed", range(6))
def test_scale_reaches_the_best_breakpoint(seed):
    _lib_or_skip()
    rng = np.random.Generator(np.random.PCG64(seed))
    D = int(rng.integers(1, 6))
    m = rng.integers(1, 12, size=D).astype(np.float64)
    limit = int(rng.integers(20, 70))
    alpha, eff, mq = wmh.choose_scale(m, limit=limit, components=D, steps=128)
    assert np.all(mq <= limit) and np.all(mq == np.ceil(alpha * m))
    best = scale.best_breakpoint(m, limit)
    got = scale.objective(alpha, m)
    assert got >= best * (1 - 1e-12)
    assert 0 < eff <= 1 + 1e-12
    assert abs(eff - float(got) * m.sum()) < 1e-9


def test_narrow_limit_and_efficiency():
    _lib_or_skip()
    rng = np.random.Generator(np.random.PCG64(9))
    m = rng.lognormal(0, 1, size=4096) * 1000.0
    a16, e16, mq16 = wmh.choose_scale(m, limit=65535)
    a32, e32, mq32 = wmh.choose_scale(m, limit=0)
    assert mq16.max() <= 65535 and mq16.max() >= 65000
    assert a32 > a16 and e32 >= e16 > 0.95


def test_bad_bounds():
    _lib_or_skip()
    with pytest.raises(wmh.WMHError):
        wmh.choose_scale(np.zeros(4))
    with pytest.raises(wmh.WMHError):
        wmh.choose_scale(np.array([1.0, -2.0]))
    with pytest.raises(wmh.WMHError):
        wmh.choose_scale(np.array([1.0, np.inf]))
