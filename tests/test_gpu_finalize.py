"""GPU: dose and batch uncertainty of raw batch tallies (Sec. II.D) against
their FP64 definitions, through gmc_finalize_tally (C ABI).

Seeded random tallies (up to 2^40 units of 2^-27 MeV per batch, a tenth of
the voxels empty, single batches empty in others) on a ragged 37 x 23 x 11
grid whose densities vary and include vacuum voxels; K = 1, 3, 7, 12 and 32
(a lane holds every batch of its voxel in registers, in arrays of 1, 4, 8,
16 and 32) and K = 40 (the general loop);
history ranges from 0 and from an offset, so that batch sizes differ.
Expected: D = sum_k T_k / (N rho V) and sigma^2 = sum_k n_k^2 (m_k - m)^2 /
(N^2 (K-1)/K), computed on the host in FP64 from the tally; the two agree
to 1e-12 relative (a few roundings apart), vacuum voxels are exactly zero,
and the tally from host memory and from device memory give the same bits.
"""
import numpy as np
import pytest

from paper_1101_1245_amd import inputs as I

pytestmark = pytest.mark.gpu
LSB = 2.0 ** -27
MEV_TO_J = 1.602176634e-13
SHAPE = (11, 23, 37)          # nz, ny, nx
VOXEL = (0.3, 0.25, 0.4)


@pytest.fixture(scope="module")
def G():
    from paper_1101_1245_amd import gpumcd
    return gpumcd


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def phantom(rng):
    ph = I.homogeneous(SHAPE[::-1], 1.0)
    rho = rng.uniform(0.2, 2.0, SHAPE).astype(np.float32)
    rho[rng.random(SHAPE) < 0.05] = 0.0
    return I.Phantom(rho=rho, mat=ph.mat, voxel=VOXEL)


def tally(rng, K):
    t = rng.integers(0, 1 << 40, size=(K,) + SHAPE, dtype=np.uint64)
    t[:, rng.random(SHAPE) < 0.1] = 0                       # voxels nothing reached
    t[rng.random((K,) + SHAPE) < 0.05] = 0                   # single empty batches
    return t


def expected(t, rho, h0, h1):
    """D and sigma of Sec. II.D from batch tallies of histories [h0, h1), history h in batch h mod K."""
    K = t.shape[0]
    n = float(h1 - h0)
    nk = np.bincount((np.arange(h0, h1, dtype=np.int64) % K), minlength=K).astype(np.float64)
    e = t.astype(np.float64) * LSB                           # MeV per batch
    rho = rho.astype(np.float64)
    vol = float(np.prod(VOXEL))
    with np.errstate(divide="ignore", invalid="ignore"):
        conv = np.where(rho > 0, MEV_TO_J / (rho * vol * 1e-3), 0.0)
    m = e.sum(axis=0) / n
    if K > 1:
        var = (nk[:, None, None, None] ** 2 * (e / nk[:, None, None, None] - m) ** 2).sum(axis=0) / (n * n * (K - 1) / K)
    else:
        var = np.zeros_like(m)
    return m * conv, np.sqrt(var) * conv


@pytest.mark.parametrize("K", [1, 3, 7, 12, 32, 40])
@pytest.mark.parametrize("h0,h1", [(0, 100_003), (12_345, 2_012_346)], ids=["from-0", "offset"])
def test_finalize_matches_definition(ctx, G, K, h0, h1):
    import torch
    rng = np.random.default_rng(1000 + K)
    ph = phantom(rng)
    t = tally(rng, K)
    print("\nfinalize K=%d on %s, histories [%d, %d)" % (K, SHAPE, h0, h1), flush=True)
    tid = ctx.load_tables((I.WATER,), I.Physics(ecut=0.7, pcut=0.01, n_batches=K))
    pid = ctx.load_phantom(ph)
    try:
        d, s, _ = ctx.finalize_tally(pid, tid, t, h0, h1)
        td = torch.from_numpy(t.view(np.int64)).to("cuda:0")
        dd, sd, _ = ctx.finalize_tally(pid, tid, td, h0, h1)
    finally:
        ctx.release(pid)
        ctx.release(tid)
    de, se = expected(t, ph.rho, h0, h1)
    assert np.array_equal(d, dd) and np.array_equal(s, sd)
    vac = ph.rho == 0
    assert not d[vac].any() and not s[vac].any()
    assert np.allclose(d, de, rtol=1e-12, atol=0.0)
    assert np.allclose(s, se, rtol=1e-12, atol=1e-12 * float(se.max()))
    if K == 1:
        assert not s.any()
