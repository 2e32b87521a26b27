"""CPU checks of the short-time-dynamics analysis (Sec. IV) on series whose
answers are fixed in closed form, and on the oracle's own series."""
import numpy as np
import pytest

from paper_1211_7275_amd import std, workloads

T = np.logspace(-1, 5, 200)


def test_gamma_is_constant_when_the_scaling_relation_holds():
    """w ~ W0 t^(zeta/z), v ~ V0 t^(-beta/(nu z)) with beta/(nu z) = 1 - zeta/z
    makes gamma = w / (t v) = W0 / V0 at every t (Sec. IV B)."""
    e = 0.128
    w2 = (0.839 * T ** (1 - e)) ** 2
    v = 0.721 * T ** (-e)
    g = std.gamma(T, w2, v)
    assert np.allclose(g, 0.839 / 0.721, rtol=1e-13)


def test_power_law_fit_is_exact_on_a_power_law():
    A, e = std.power_law_fit(T, 3.5 * T ** -0.25, 1.0, 1e4)
    assert A == pytest.approx(3.5, rel=1e-12)
    assert e == pytest.approx(-0.25, abs=1e-12)


@pytest.mark.parametrize("A,e,tc,alpha", [(0.721, -0.128, 0.110, 0.715),   # v, RB (Sec. IV D)
                                          (0.839, 0.872, 0.485, 0.712),    # w, RB
                                          (0.53, -0.128, 0.382, 0.927)])   # v, RF
def test_corrected_fit_recovers_its_parameters(A, e, tc, alpha):
    y = A * T ** e * (1 + (T / tc) ** -alpha)
    fit = std.corrected_fit(T, y, t_mic=1.0)
    assert fit["A"] == pytest.approx(A, rel=1e-6)
    assert fit["e"] == pytest.approx(e, abs=1e-7)
    assert fit["t_c"] == pytest.approx(tc, rel=1e-5)
    assert fit["alpha"] == pytest.approx(alpha, rel=1e-6)


def test_gamma_fit_recovers_its_parameters():
    g = 1.143 * (1 + (T / 0.142) ** -0.56)
    fit = std.gamma_fit(T, g, t_mic=1.0)
    assert fit["G0"] == pytest.approx(1.143, rel=1e-6)
    assert fit["t_g"] == pytest.approx(0.142, rel=1e-5)
    assert fit["alpha_g"] == pytest.approx(0.56, rel=1e-6)


def test_window_exponents_show_the_positive_bias_at_early_times():
    """Procedure (c): pure power-law fits on [t0, 4 t0] of the corrected velocity
    overestimate beta/(nu z) at small t0 and converge to it as t0 grows."""
    v = 0.721 * T ** -0.128 * (1 + (T / 0.110) ** -0.715)
    t0s = np.array([1.0, 10.0, 100.0, 1000.0, 10000.0])
    ex = -std.window_exponents(T, v, t0s)
    assert np.all(np.diff(ex) < 0)
    assert ex[0] > 0.2
    assert ex[-1] == pytest.approx(0.128, abs=2e-4)


def _synthetic_v(f, fc, t):
    x = (f - fc) * np.sqrt(t)
    return t ** -0.128 * (np.exp(x) if f < fc else 1 + x)


def test_bracket_fc_on_synthetic_curves():
    drives = np.round(np.arange(0.90, 1.101, 0.02), 2)
    fc = 1.013
    v = np.array([_synthetic_v(f, fc, T[50:]) for f in drives])
    f_lo, f_hi, signs = std.bracket_fc(drives, T[50:], v)
    assert (f_lo, f_hi) == (1.0, 1.02)
    assert np.array_equal(signs, np.where(drives > fc, 1, -1))
    # exactly critical: v ~ t^(-0.128) is on the boundary; slightly faster decay dies
    assert std.classify_drive(T, T ** -0.12) == 1
    assert std.classify_drive(T, T ** -0.14) == -1
    # a pinned line (v down to rounding) dies even if its last values are flat
    assert std.classify_drive(T, np.full(T.size, 1e-7)) == -1


def test_bracket_fc_on_oracle_series(oracle):
    """A drive well below and one well above the threshold of a small RF chain,
    evolved by the oracle: the first dies, the second saturates."""
    meas = workloads.log_steps(20_000, 40)
    drives = np.array([0.3, 2.0])
    v = []
    for f in drives:
        p = workloads.custom(0, [256] * 2, f, 20_000, meas, workloads.SEED_BASE + 60,
                             disorder_id=[0, 1])
        v.append(oracle.run(p)["v"].mean(0))
    f_lo, f_hi, signs = std.bracket_fc(drives, meas * 0.05, np.array(v))
    assert (f_lo, f_hi) == (0.3, 2.0)


def test_exponents_of_a_corrected_critical_decay():
    """The exponent report of one drive: windowed estimates converge to the
    exponents of corrected power laws, the corrected fits return them."""
    e = 0.128
    v = 0.721 * T ** -e * (1 + (T / 0.110) ** -0.715)
    w = 0.839 * T ** (1 - e) * (1 + (T / 0.485) ** -0.712)
    r = std.exponents(T, v, w ** 2)
    assert r["beta_over_nu_z"][-1] == pytest.approx(e, abs=2e-4)
    assert r["one_minus_zeta_over_z"][-1] == pytest.approx(e, abs=5e-4)
    assert r["corrected_beta_over_nu_z"] == pytest.approx(e, abs=1e-6)
    assert r["corrected_one_minus_zeta_over_z"] == pytest.approx(e, abs=1e-6)
