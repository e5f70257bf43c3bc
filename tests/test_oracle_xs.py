"""Pins of the oracle's closed-form cross sections and stopping powers.

Each closed form in the oracle is an integral of a differential cross section
(Sec. II.A, II.B, Eqs. 2, 5, 6).  The tests integrate the differential form
numerically (scipy quad), written here in a different variable where one is
natural, and compare; limits and identities that the mathematics fixes are
checked too.  A dropped term, a wrong sign or a wrong limit in a closed form
fails one of them.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from paper_1101_1245_amd.inputs import BONE, SOFT_TISSUE, WATER

MC2 = 0.51099895
RE = 2.8179403262e-13
NA = 6.02214076e23
ALPHA = 1 / 137.035999084
MATS = [WATER, BONE, SOFT_TISSUE]


def kn_dcs_domega(k, mu):
    """Klein-Nishina per electron, d sigma / d Omega (cm^2/sr), cos theta = mu."""
    p = 1.0 / (1.0 + k * (1.0 - mu))
    return 0.5 * RE ** 2 * p * p * (p + 1.0 / p - (1.0 - mu * mu))


@pytest.mark.parametrize("e", [0.001, 0.03, 0.2, 1.0, 6.0, 15.0, 30.0])
def test_compton_total_is_integral_of_kn(oracle, e):
    k = e / MC2
    sig = 2 * np.pi * quad(lambda mu: kn_dcs_domega(k, mu), -1, 1, epsabs=0, epsrel=1e-12)[0]
    for m in MATS:
        want = NA * m.z_over_a * sig
        assert oracle.xs(m, "mu_C", [e])[0] == pytest.approx(want, rel=1e-9)


def test_compton_thomson_limit(oracle):
    thomson = 8 * np.pi / 3 * RE ** 2
    got = oracle.xs(WATER, "mu_C", [1e-3])[0] / (NA * WATER.z_over_a)
    k = 1e-3 / MC2
    assert got == pytest.approx(thomson * (1 - 2 * k), rel=2e-5)   # first-order KN correction


def test_photoelectric_crossing_and_scaling(oracle):
    # C_pe is fixed by the crossing of water's photoelectric and Compton terms at 26 keV
    assert oracle.xs(WATER, "mu_pe", [0.026])[0] == pytest.approx(oracle.xs(WATER, "mu_C", [0.026])[0], rel=1e-7)
    e = np.array([0.01, 0.1, 1.0])
    w = oracle.xs(WATER, "mu_pe", e)
    assert w[0] / w[1] == pytest.approx(1000.0, rel=1e-12)          # E^-3
    b = oracle.xs(BONE, "mu_pe", e)
    ratio = (BONE.z_over_a * BONE.z_eff ** 3) / (WATER.z_over_a * WATER.z_eff ** 3)  # per-atom Z^4/A
    assert b[2] / w[2] == pytest.approx(ratio, rel=1e-12)


def test_pair_threshold_and_shape(oracle):
    e = np.array([0.9, 2 * MC2, 2 * MC2 * (1 + 1e-9), 1.5, 10.0])
    v = oracle.xs(WATER, "mu_pair", e)
    assert v[0] == 0.0 and v[1] == 0.0
    assert 0.0 <= v[2] < 1e-20 and v[3] > 0 and v[4] > v[3]
    # Z(Z+1)/A scaling between materials at fixed energy
    r = oracle.xs(BONE, "mu_pair", [10.0])[0] / oracle.xs(WATER, "mu_pair", [10.0])[0]
    want = BONE.z_over_a * (BONE.z_eff + 1) / (WATER.z_over_a * (WATER.z_eff + 1))
    assert r == pytest.approx(want, rel=1e-12)
    # high-energy slope: d mu / d ln E -> the log coefficient as (1-2/k)^3 -> 1
    e1, e2 = 1e7, 2e7
    a, b = oracle.xs(WATER, "mu_pair", [e1, e2])
    coef = NA * WATER.z_over_a * (WATER.z_eff + 1) * ALPHA * RE ** 2 * 2.0
    assert (b - a) / np.log(2) == pytest.approx(coef, rel=1e-3)


def test_attenuation_sanity_vs_tabulated_water(oracle):
    # Sanity against tabulated water attenuation without coherent scattering
    # (NIST XCOM, approximate): 1 MeV 0.0707, 6 MeV 0.0277, 15 MeV 0.0194 cm^2/g.
    e = np.array([1.0, 6.0, 15.0])
    tot = sum(oracle.xs(WATER, w, e) for w in ("mu_C", "mu_pe", "mu_pair"))
    assert np.allclose(tot, [0.0707, 0.0277, 0.0194], rtol=0.03)


def moller_dcs_dw(t, w):
    """Moller d sigma / dW per electron / (2 pi r_e^2 mc^2 / beta^2), energy transfer W."""
    tau = t / MC2
    g = tau + 1
    return (1 / w ** 2 + 1 / (t - w) ** 2 + (tau / g) ** 2 / t ** 2
            - (2 * tau + 1) / (g ** 2 * w * (t - w)))


def beta2(t):
    g = 1 + t / MC2
    return 1 - 1 / g ** 2


@pytest.mark.parametrize("t", [0.5, 1.0, 3.0, 15.0, 25.0])
@pytest.mark.parametrize("kcut", [0.01, 0.2, 0.7])
def test_moller_cross_section_and_hard_loss(oracle, t, kcut):
    for m in (WATER, BONE):
        sig = oracle.xs(m, "Sigma_M", [t], kcut=kcut)[0]
        eh = oracle.xs(m, "E_M_hard", [t], kcut=kcut)[0]
        if t <= 2 * kcut:
            assert sig == 0.0 and eh == 0.0
            continue
        pref = 2 * np.pi * RE ** 2 * MC2 / beta2(t) * NA * m.z_over_a
        s_num = pref * quad(lambda w: moller_dcs_dw(t, w), kcut, t / 2, epsrel=1e-12, limit=200)[0]
        e_num = pref * quad(lambda w: w * moller_dcs_dw(t, w), kcut, t / 2, epsrel=1e-12, limit=200)[0]
        assert sig == pytest.approx(s_num, rel=1e-8)
        assert eh == pytest.approx(e_num, rel=1e-8)
        # restricted collision stopping power plus the hard part is the full Bethe value
        lcol = oracle.xs(m, "L_col", [t], kcut=kcut)[0]
        assert lcol + e_num == pytest.approx(oracle.xs(m, "S_col", [t])[0], rel=1e-9)


def test_restricted_equals_full_at_half(oracle):
    t = np.array([0.3, 1.0, 10.0])
    for i, tt in enumerate(t):
        assert oracle.xs(WATER, "L_col", [tt], kcut=tt / 2)[0] == pytest.approx(
            oracle.xs(WATER, "S_col", [tt])[0], rel=1e-12)


def test_collision_stopping_sanity(oracle):
    # NIST ESTAR water collision stopping powers include the density effect
    # (1 MeV: 1.849, 10 MeV: 1.968 MeV cm^2/g); without it the Bethe value is
    # higher by the density correction, which grows with energy (about 1% at
    # 1 MeV and about 13% at 10 MeV in water).
    s = oracle.xs(WATER, "S_col", [1.0, 10.0])
    assert 1.849 < s[0] < 1.849 * 1.03
    assert 1.968 * 1.05 < s[1] < 1.968 * 1.16
    # minimum of dE/dx near 1.5 - 2 MeV for electrons in water
    e = np.geomspace(0.1, 20, 400)
    v = oracle.xs(WATER, "S_col", e)
    assert 0.8 < e[np.argmin(v)] < 3.0


def brems_dcs_dk(t, k, x0):
    e = t + MC2
    y = k / e
    return (4 / 3 - 4 * y / 3 + y * y) / (k * x0)


def x0_of(m):
    a = m.z_eff / m.z_over_a
    return 716.4 * a / (m.z_eff * (m.z_eff + 1) * np.log(287 / np.sqrt(m.z_eff)))


@pytest.mark.parametrize("t", [0.005, 0.5, 2.0, 15.0])
@pytest.mark.parametrize("kc", [0.01, 0.05])
def test_brems_cross_section_and_losses(oracle, t, kc):
    for m in (WATER, BONE):
        x0 = x0_of(m)
        sig = oracle.xs(m, "Sigma_B", [t], kc=kc)[0]
        lrad = oracle.xs(m, "L_rad", [t], kc=kc)[0]
        srad = oracle.xs(m, "S_rad", [t])[0]
        if t <= kc:
            assert sig == 0.0
        else:
            assert sig == pytest.approx(quad(lambda k: brems_dcs_dk(t, k, x0), kc, t, epsrel=1e-12)[0], rel=1e-9)
        kk = min(kc, t)
        assert lrad == pytest.approx(quad(lambda k: k * brems_dcs_dk(t, k, x0), 0, kk, epsrel=1e-12)[0], rel=1e-9)
        assert srad == pytest.approx(quad(lambda k: k * brems_dcs_dk(t, k, x0), 0, t, epsrel=1e-12)[0], rel=1e-9)


def test_radiation_length_values(oracle):
    # high-energy limit of the radiative stopping power: S_rad/E -> (4/3 - 2/3 + 1/3)/X0 = 1/X0
    for m in MATS:
        t = 1e5
        srad = oracle.xs(m, "S_rad", [t])[0]
        assert srad / (t + MC2) == pytest.approx(1 / x0_of(m), rel=1e-4)
    assert x0_of(WATER) == pytest.approx(32.911, rel=1e-4)


def screened_rutherford_transport(m, t, eta):
    """sigma_1 per electron-atom scaling: 2 pi Z(Z+1) r_e^2 (mc^2/(beta pc))^2 int w/(w+2 eta)^2 dw."""
    pc = np.sqrt(t * (t + 2 * MC2))
    beta = pc / (t + MC2)
    pref = 2 * np.pi * m.z_eff * (m.z_eff + 1) * RE ** 2 * (MC2 / (beta * pc)) ** 2
    integ = quad(lambda w: w / (w + 2 * eta) ** 2, 0, 2, epsrel=1e-12, points=[2 * eta, 20 * eta], limit=400)[0]
    return pref * integ * NA / (m.z_eff / m.z_over_a)


@pytest.mark.parametrize("t", [0.05, 1.0, 15.0])
def test_transport_mean_free_path(oracle, t):
    for m in (WATER, BONE):
        eta = oracle.xs(m, "eta", [t])[0]
        pc = np.sqrt(t * (t + 2 * MC2))
        beta = pc / (t + MC2)
        # Moliere screening with the Thomas-Fermi radius 0.885 a0 Z^-1/3
        want_eta = 0.25 * (ALPHA * MC2 / pc * m.z_eff ** (1 / 3) / 0.885) ** 2 * (1.13 + 3.76 * (ALPHA * m.z_eff / beta) ** 2)
        assert eta == pytest.approx(want_eta, rel=1e-12)
        got = oracle.xs(m, "inv_lambda1", [t])[0]
        assert got == pytest.approx(screened_rutherford_transport(m, t, eta), rel=1e-7)


def test_csda_range_sanity(oracle):
    # Restricted and unrestricted totals are positive and ordered
    e = np.geomspace(0.01, 30, 200)
    for m in MATS:
        L = oracle.xs(m, "L", e, kcut=0.2, kc=0.01)
        S = oracle.xs(m, "S_col", e) + oracle.xs(m, "S_rad", e)
        assert np.all(L > 0) and np.all(L <= S * (1 + 1e-12))


def test_majorants_bound_every_energy(oracle):
    from paper_1101_1245_amd.inputs import Physics, z_slabs
    ph = z_slabs(8, 1.0, [(3.0, 0, 1.0), (5.0, 1, 1.85), (12.0, 2, 0.26)])
    mats = (WATER, BONE, SOFT_TISSUE)
    phys = Physics(ecut=0.2, pcut=0.01)
    mu_hat, sig_hat = oracle.majorants(mats, ph, phys)
    n = oracle.grid_size()
    grid = 1e-3 * np.exp(np.arange(n) * np.log(32e3) / (n - 1))
    e = np.geomspace(1.0001e-3, 31.99, 20000)
    b = np.clip(np.floor(np.log(e / 1e-3) * (n - 1) / np.log(32e3)).astype(int), 0, n - 2)
    assert np.all(grid[b] <= e * (1 + 1e-12)) and np.all(e <= grid[b + 1] * (1 + 1e-12))
    rmax = {0: 1.0, 1: 1.85, 2: 0.26}
    for mi, r in rmax.items():
        mu = r * sum(oracle.xs(mats[mi], w, e) for w in ("mu_C", "mu_pe", "mu_pair"))
        assert np.all(mu <= mu_hat[b])
        sg = r * (oracle.xs(mats[mi], "Sigma_M", e, kcut=0.2) + oracle.xs(mats[mi], "Sigma_B", e, kc=0.01))
        # every energy below the bin's upper edge is bounded by the bin's Sigma_hat
        run = np.maximum.accumulate(sg)
        assert np.all(run <= sig_hat[b])
    # the majorant is tight to within the 1e-3 margin plus the bin variation
    assert np.max(mu_hat[b] / (1.85 * sum(oracle.xs(BONE, w, e) for w in ("mu_C", "mu_pe", "mu_pair")))) < 1.05
