import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O.build()
    return O


@pytest.fixture(scope="session")
def batched_run():
    """A plain GPU run through the raw-tally entry points: (dose, sigma, stats,
    (per-batch doses, batch sizes)) -- the dose and sigma equal gmc_run_beam's
    bit for bit; the batches feed the z-test's mean bound."""
    import numpy as np
    from paper_1101_1245_amd import evaluate as E

    def run(ctx, pid, tid, source, n, seed, phantom):
        t, st = ctx.run_beam_tally(pid, tid, source, n, seed)
        d, s, _ = ctx.finalize_tally(pid, tid, t, 0, n)
        dk, nk = E.batch_doses(t.astype(np.float64) * E.LSB_MEV, phantom.rho, phantom.voxel, n)
        return d, s, st, (dk, nk)
    return run


def oracle_batches(res, phantom, n):
    """Per-batch doses of an oracle run with batches (history h in batch h mod K)."""
    from paper_1101_1245_amd import evaluate as E
    return E.batch_doses(res.eb, phantom.rho, phantom.voxel, n)
