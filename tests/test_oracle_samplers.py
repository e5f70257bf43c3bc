"""KS pins of the oracle's samplers against their differential cross sections.

For every sampled quantity the test integrates the differential cross section
numerically (written here in the natural variable: cos theta for angles, the
energy transfer for Moller and bremsstrahlung) into a CDF and runs a
Kolmogorov-Smirnov test on 2e5 samples from fixed seeds (Sec. II.A: Compton,
photoelectric, pair; Sec. II.B.1: Moller, bremsstrahlung; Sec. II.B.2:
multiple-scattering shape).
"""
import numpy as np
import pytest
from scipy import stats
from scipy.integrate import quad

MC2 = 0.51099895
N = 200000
P_MIN = 1e-3


def numeric_cdf(f, grid):
    seg = np.array([quad(f, a, b, epsrel=1e-10, limit=200)[0] for a, b in zip(grid[:-1], grid[1:])])
    c = np.concatenate([[0.0], np.cumsum(seg)])
    c /= c[-1]
    return lambda x: np.interp(x, grid, c)


def beta_gamma(t):
    g = 1 + t / MC2
    return np.sqrt(1 - 1 / g ** 2), g


def dense_grid(a, b, peak, width, n=3000):
    """Grid on [a, b] dense near ``peak`` (scale ``width``)."""
    u = np.linspace(-1, 1, n)
    lo = np.arcsinh((a - peak) / width)
    hi = np.arcsinh((b - peak) / width)
    g = peak + width * np.sinh(lo + (hi - lo) * (u + 1) / 2)
    g[0], g[-1] = a, b
    return np.unique(g)


@pytest.mark.parametrize("e", [0.02, 0.5, 2.0, 15.0])
def test_klein_nishina_angle(oracle, e):
    k = e / MC2
    eps, cost = oracle.sample("kn", e, seed=11, count=N)

    def dcs(mu):
        p = 1.0 / (1.0 + k * (1.0 - mu))
        return p * p * (p + 1.0 / p - (1.0 - mu * mu))

    cdf = numeric_cdf(dcs, dense_grid(-1, 1, 1.0, min(1.0, 2.0 / k)))
    assert stats.kstest(cost, cdf).pvalue > P_MIN
    # the energy fraction follows from the angle (Compton kinematics)
    assert np.allclose(eps, 1.0 / (1.0 + k * (1.0 - cost)), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("t", [0.01, 0.1, 1.0, 10.0])
def test_sauter_photoelectron_angle(oracle, t):
    beta, g = beta_gamma(t)
    cost = oracle.sample("sauter", t, seed=12, count=N)
    assert np.all(cost >= -1.0) and np.all(cost <= 1.0)

    def dcs(mu):
        x = 1 - beta * mu
        return (1 - mu * mu) / x ** 4 * (1 + 0.5 * g * (g - 1) * (g - 2) * x)

    width = max(1e-6, 1 - beta)
    cdf = numeric_cdf(dcs, dense_grid(-1, 1, 1.0, width * 4))
    assert stats.kstest(cost, cdf).pvalue > P_MIN


@pytest.mark.parametrize("t", [0.0, 0.3, 3.0, 12.0])
def test_pair_electron_angle(oracle, t):
    beta, g = beta_gamma(t)
    cost = oracle.sample("pair", t, seed=13, count=N)
    assert np.all(np.abs(cost) <= 1.0 + 1e-12)
    cdf = numeric_cdf(lambda mu: (1 - beta * mu) ** -2, dense_grid(-1, 1, 1.0, max(1e-6, 2 * (1 - beta))))
    assert stats.kstest(cost, cdf).pvalue > P_MIN


@pytest.mark.parametrize("t,kcut", [(1.0, 0.2), (5.0, 0.7), (15.0, 0.7), (20.0, 0.01)])
def test_moller_energy_transfer(oracle, t, kcut):
    tau = t / MC2
    g = tau + 1
    eps = oracle.sample("moller", t, kcut, seed=14, count=N)
    assert np.all(eps >= kcut / t) and np.all(eps <= 0.5)

    def dcs(w):   # d sigma / dW up to constants
        return 1 / w ** 2 + 1 / (t - w) ** 2 + (tau / g) ** 2 / t ** 2 - (2 * tau + 1) / (g ** 2 * w * (t - w))

    grid = np.geomspace(kcut, t / 2, 3000)
    cdf = numeric_cdf(dcs, grid)
    assert stats.kstest(eps * t, cdf).pvalue > P_MIN


@pytest.mark.parametrize("t,kc", [(0.5, 0.01), (2.0, 0.01), (15.0, 0.01), (20.0, 0.2)])
def test_brems_photon_energy(oracle, t, kc):
    e = t + MC2
    k = oracle.sample("brems", t, kc, seed=15, count=N)
    assert np.all(k >= kc) and np.all(k <= t)
    cdf = numeric_cdf(lambda x: (4 / 3 - 4 * x / (3 * e) + (x / e) ** 2) / x, np.geomspace(kc, t, 3000))
    assert stats.kstest(k, cdf).pvalue > P_MIN


@pytest.mark.parametrize("g1", [1e-6, 1e-3, 0.05, 0.4, 0.9, 0.9995])
def test_wentzel_shape_and_first_moment(oracle, g1):
    cost = oracle.sample("wentzel", g1, seed=16, count=N)
    w = 1 - cost
    if g1 >= 0.9999:
        assert stats.kstest(w / 2, "uniform").pvalue > P_MIN
        return
    a = oracle.ms_screening_A(g1)
    # the screening parameter reproduces the first moment: int w p(w) = G1,
    # p(w) ~ 1/(2A + w)^2 on [0, 2]
    pts = [min(2.0, 2 * a), min(2.0, 20 * a)]
    num = quad(lambda x: x / (2 * a + x) ** 2, 0, 2, points=pts, epsrel=1e-12, limit=400)[0]
    den = quad(lambda x: 1 / (2 * a + x) ** 2, 0, 2, points=pts, epsrel=1e-12, limit=400)[0]
    assert num / den == pytest.approx(g1, rel=1e-9)
    cdf = numeric_cdf(lambda x: 1 / (2 * a + x) ** 2, dense_grid(0, 2, 0.0, 2 * a))
    assert stats.kstest(w, cdf).pvalue > P_MIN
    # sample mean within 5 standard errors
    assert abs(w.mean() - g1) < 5 * w.std() / np.sqrt(N) + 1e-12


def test_wentzel_limits(oracle):
    assert oracle.sample("wentzel", 0.0, count=10).tolist() == [1.0] * 10
    a_small = oracle.ms_screening_A(1e-12)
    assert 0 < a_small < 1e-12
    a_big = oracle.ms_screening_A(0.99)
    # 1 - G1 -> 1/(3A) for large A
    assert 1 / (3 * a_big) == pytest.approx(0.01, rel=0.2)


def test_rotation_geometry(oracle):
    rng = np.random.default_rng(3)
    for _ in range(500):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        if rng.uniform() < 0.1:
            d = np.array([0.0, 0.0, rng.choice([-1.0, 1.0])])
        cost = rng.uniform(-1, 1)
        phi = rng.uniform(0, 2 * np.pi)
        o = oracle.rotate(d, cost, phi)
        assert np.linalg.norm(o) == pytest.approx(1.0, abs=1e-14)
        assert np.dot(o, d) == pytest.approx(cost, abs=1e-12)
        # phi and phi + pi give mirror images about d
        o2 = oracle.rotate(d, cost, phi + np.pi)
        assert np.allclose(o + o2, 2 * cost * d, atol=1e-12)
    # azimuth is uniform around d: the mean of many rotated vectors is cos(theta) d
    d = np.array([0.6, 0.0, 0.8])
    phis = np.linspace(0, 2 * np.pi, 4096, endpoint=False)
    m = np.mean([oracle.rotate(d, 0.3, p) for p in phis], axis=0)
    assert np.allclose(m, 0.3 * d, atol=1e-12)
