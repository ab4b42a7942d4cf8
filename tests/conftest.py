import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.lib()
    return oracle


def _support_band(gr, ga, full_r, full_a, full_abs, M, rel=1e-12):
    """Truncated sigma of the fast (unordered-sum) mode against the oracle's
    untruncated sigma (full_r, full_a, with per-entry sums of |terms|): the
    kept count is min(M, nonzero); on the common support the values agree to
    1e-12 of the per-entry absolute sum; the supports may differ only on
    entries whose magnitude lies within rel of the M-th magnitude tau (ties
    in exact arithmetic that rounding decides).  Returns the number of
    differing entries."""
    import numpy as np

    import oracle

    kr, ka = oracle.topm(full_r, full_a, M)
    assert len(gr) == len(kr)
    if len(kr) == 0:
        return 0
    tau = float(np.abs(ka).min())
    pos = np.searchsorted(full_r, gr)
    assert np.all(pos < len(full_r)) and np.array_equal(full_r[pos], gr), "a kept entry is not in sigma"
    assert np.all(np.abs(ga - full_a[pos]) <= 1e-12 * full_abs[pos])
    diff = np.setxor1d(gr, kr)
    if len(diff):
        dpos = np.searchsorted(full_r, diff)
        mags = np.abs(full_a[dpos])
        assert np.all(np.abs(mags - tau) <= rel * tau), (diff, mags, tau)
    return int(len(diff))


@pytest.fixture(scope="session")
def support_band():
    return _support_band
