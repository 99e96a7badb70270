"""Host logic of the finite-size-scaling driver, checked against closed forms
and synthetic data of a known scaling form (Sec. 3.1, Eqs. 2-4), and its
moment ratio against the oracle's definition of U on oracle records."""
import numpy as np
import pytest

import oracle
from paper_1612_08312_amd import fss, workloads


def test_jackknife_of_a_mean_is_the_standard_error():
    rng = np.random.default_rng(5)
    v = rng.normal(size=7)
    est, err = fss.jackknife(v, np.mean)
    assert est == pytest.approx(np.mean(v), rel=1e-15)
    assert err == pytest.approx(np.std(v, ddof=1) / np.sqrt(len(v)), rel=1e-12)


def test_jackknife_of_a_ratio_matches_the_delta_method_for_small_noise():
    """For f = mean(a)/mean(b) with tiny noise the jackknife error equals the
    standard error of the linearised f."""
    rng = np.random.default_rng(6)
    R = 400
    a = 2.0 + 1e-4 * rng.normal(size=R)
    b = 4.0 + 1e-4 * rng.normal(size=R)
    v = np.stack([a, b], axis=1)
    _, err = fss.jackknife(v, lambda x: x[:, 0].mean() / x[:, 1].mean())
    g = a / 4.0 - 2.0 * b / 16.0  # linearised f: df = da / b - a db / b^2 at (2, 4)
    delta = np.std(g, ddof=1) / np.sqrt(R)
    assert err == pytest.approx(delta, rel=1e-3)


def test_line_root_and_crossing_of_two_lines():
    T = np.linspace(4.0, 4.4, 9)
    assert fss.line_root(T, 3.0 * (T - 4.2139)) == pytest.approx(4.2139, abs=1e-12)
    u1 = 1.5 - 2.0 * (T - 4.21)
    u2 = 1.5 - 5.0 * (T - 4.21)
    assert fss.crossing(T, u1, u2) == pytest.approx(4.21, abs=1e-12)
    # weights do not move the root of exact data
    w = np.linspace(0.01, 0.1, 9)
    assert fss.crossing(T, u1, u2, w, w[::-1]) == pytest.approx(4.21, abs=1e-12)


def scaling_data(tc, nu, bn, Ls, temps, runs, noise, seed):
    """Per-run means [L][T][run][2] whose U and <m^2> follow Eqs. 3-4 exactly
    (up to noise): U = f1(x), <m^2> = Lp^(-2 bn) f2(x), x = t Lp^(1/nu)."""
    rng = np.random.default_rng(seed)
    f1 = lambda x: 2.0 + np.tanh(0.3 * x)
    f2 = lambda x: 0.6 * np.exp(-0.3 * x)
    out = np.zeros((len(Ls), len(temps), runs, 2))
    T = np.asarray(temps)
    for li, L in enumerate(Ls):
        lp = fss.linear_size(L)
        x = (T - tc) / tc * lp ** (1.0 / nu)
        m2 = lp ** (-2.0 * bn) * f2(x)
        m4 = f1(x) * m2 ** 2
        for r in range(runs):
            out[li, :, r, 0] = m2 * (1 + noise * rng.normal(size=len(T)))
            out[li, :, r, 1] = m4 * (1 + noise * rng.normal(size=len(T)))
    return out


def test_estimates_form_the_ratio_of_run_averaged_moments():
    rm = scaling_data(4.2, 0.63, 0.52, (8, 16), np.linspace(4.19, 4.21, 5), 4, 1e-3, 1)
    U, dU, m2, dm2 = fss.estimates(rm)
    np.testing.assert_allclose(m2, rm[..., 0].mean(axis=-1), rtol=1e-14)
    np.testing.assert_allclose(U, rm[..., 1].mean(axis=-1) / rm[..., 0].mean(axis=-1) ** 2, rtol=1e-14)
    np.testing.assert_allclose(dm2, rm[..., 0].std(axis=-1, ddof=1) / 2.0, rtol=1e-10)
    assert np.all(dU > 0)


def test_collapse_quality_is_zero_for_exact_collapse_and_grows_off_it():
    Ls = (32, 48, 64, 96)
    temps = fss.default_temperatures(workloads.ISING)
    rm = scaling_data(4.21394, 0.629, 0.52, Ls, temps, 3, 0.0, 2)
    U, _, _, _ = fss.estimates(rm)
    dU = np.full_like(U, 1e-2)
    # exact data: only the linear-interpolation error of a smooth curve
    q0 = fss.collapse_quality(*fss._scaled(temps, Ls, 4.21394, 0.629, U, dU))
    q1 = fss.collapse_quality(*fss._scaled(temps, Ls, 4.2145, 0.629, U, dU))
    q2 = fss.collapse_quality(*fss._scaled(temps, Ls, 4.21394, 0.70, U, dU))
    assert q0 < 0.1
    assert q1 > 50 * q0 and q2 > 50 * q0


def test_collapse_fit_recovers_the_scaling_parameters():
    """Noisy data of a known scaling form: the fitted T_c, nu and beta/nu are
    within a few jackknife errors of the values that generated it, and the
    crossings of successive sizes sit at T_c."""
    tc, nu, bn = 4.21394, 0.629, 0.520
    Ls = (32, 48, 64, 96)
    temps = tuple(fss.default_temperatures(workloads.ISING))
    rm = scaling_data(tc, nu, bn, Ls, temps, 5, 2e-3, 3)
    res = fss.analyse(temps, Ls, rm, 4.2140, 0.65)
    assert abs(res["Tc"] - tc) < max(4 * res["dTc"], 2e-6)
    assert abs(res["nu"] - nu) < max(4 * res["dnu"], 2e-3)
    assert abs(res["beta_over_nu"] - bn) < max(4 * res["dbeta_over_nu"], 2e-3)
    assert res["quality_U"] < 5.0
    for c in res["crossings"]:
        assert abs(c["T"] - tc) < max(5 * c["dT"], 1e-5)
    # the linear measure is reported beside the default one, with its own errors
    lin = res["collapse_linear"]
    assert res["collapse_order"] == 2
    assert set(lin) == {"Tc", "dTc", "nu", "dnu", "beta_over_nu", "dbeta_over_nu", "quality_U", "quality_m2"}
    assert abs(lin["Tc"] - tc) < max(6 * lin["dTc"], 5e-6)


def test_fit_detects_a_wrong_starting_point():
    """Started away from the truth, the fit still lands on it."""
    Ls = (32, 64)
    temps = np.linspace(4.209, 4.219, 41)  # dense: no interpolation bias
    rm = scaling_data(4.2139, 0.63, 0.5, Ls, temps, 3, 0.0, 4)
    U, _, _, _ = fss.estimates(rm)
    dU = np.full_like(U, 1e-4)
    t, n, _ = fss.fit_tc_nu(temps, Ls, U, dU, 4.2125, 0.70)
    assert t == pytest.approx(4.2139, abs=5e-6)
    assert n == pytest.approx(0.63, abs=2e-3)


def test_protocol_members_and_default_window():
    p = fss.Protocol(model=workloads.XY, Ls=(8, 12), temps=(2.0, 2.1, 2.2), runs=5, seed=10)
    m = p.members()
    assert len(m) == 2 * 3 * 5
    assert len({s for (_, _, _, s) in m}) == len(m)
    assert p.sweeps_per_member() == 210_000  # Sec. 2: 10^4 discarded + 2 x 10^5 measured
    t = fss.default_temperatures(workloads.HEISENBERG)
    assert len(t) == 13 and t[6] == pytest.approx(workloads.TC[workloads.HEISENBERG], rel=1e-15)
    assert fss.linear_size(32) == pytest.approx(32 * 16 ** (1 / 3), rel=1e-15)


def test_run_averaged_ratio_equals_the_oracle_binder_of_pooled_records():
    """With equal run lengths, U from run-averaged moments is the oracle's
    U = <m^4>/<m^2>^2 (Eq. 2) over the pooled measured records."""
    L, T, discard, measure, runs = 2, 4.2139, 20, 200, 3
    p = fss.Protocol(model=workloads.ISING, Ls=(L,), temps=(T,), discard=discard,
                     measure=measure, runs=runs, seed=40)
    data = fss.RunData(protocol=p)
    pooled = []
    for (L_, ti, r, s) in p.members():
        o = oracle.Oracle(L=L_, model=workloads.ISING, T=T, seed=s, start=workloads.RANDOM)
        rec = o.sweep(discard + measure)
        keep = rec[discard:]
        pooled.append(keep)
        data.m2.setdefault(L_, {}).setdefault(ti, {})[r] = keep["m2"]
        data.m4.setdefault(L_, {}).setdefault(ti, {})[r] = keep["m4"]
    U, _, _, _ = fss.estimates(fss.run_means(data))
    want = oracle.binder(np.concatenate(pooled))
    assert U[0, 0] == pytest.approx(want, rel=1e-12)


def test_universal_metric_factors_are_recovered():
    """Two lattices whose data follow the universal forms of Sec. 3.4 with
    known metric factors (simple cubic D1 = D2 = 1, pyrochlore D1 = 0.96,
    D2 = 0.91) and their own T_c: the fit returns the pyrochlore factors."""
    nu, bn = 0.672, 0.515
    f1 = lambda x: 2.0 + np.tanh(0.3 * x)
    f2 = lambda x: 0.6 * np.exp(-0.3 * x)
    rng = np.random.default_rng(12)

    def scan(lattice, Ls, tc, d1, d2, noise=1e-3, runs=5):
        temps = tuple(float(t) for t in tc * (1 + np.linspace(-1.2e-3, 1.2e-3, 13)))
        rm = np.zeros((len(Ls), len(temps), runs, 2))
        T = np.asarray(temps)
        for li, L in enumerate(Ls):
            lp = fss.linear_size(L, lattice)
            x = d1 * (T - tc) / tc * lp ** (1 / nu)
            m2 = d2 * lp ** (-2 * bn) * f2(x)
            m4 = f1(x) * m2 ** 2
            for r in range(runs):
                rm[li, :, r, 0] = m2 * (1 + noise * rng.normal(size=len(T)))
                rm[li, :, r, 1] = m4 * (1 + noise * rng.normal(size=len(T)))
        return dict(temps=temps, L=list(Ls), Tc=tc, run_means=rm.tolist())

    pyro = scan("pyro", (32, 48, 64), 2.0285, 0.96, 0.91)
    sc = scan("sc", (64, 96, 128), 2.20182, 1.0, 1.0)
    res = fss.universal_factors(pyro, sc, nu, bn)
    assert abs(res["D1"] - 0.96) < max(4 * res["dD1"], 0.01)
    assert abs(res["D2"] - 0.91) < max(4 * res["dD2"], 0.01)
    assert res["quality_U"] < 5 and res["quality_m2"] < 5
    # the same data with the factors dropped collapse far worse
    wrong = dict(pyro)
    rm = np.asarray(pyro["run_means"]).copy()
    rm[..., 0] /= 0.91
    rm[..., 1] /= 0.91 ** 2
    wrong["run_means"] = rm.tolist()
    assert fss.universal_factors(wrong, sc, nu, bn)["D2"] == pytest.approx(1.0, abs=0.02)


def test_simple_cubic_linear_size():
    assert fss.linear_size(64, "sc") == 64.0
    assert fss.linear_size(64) == pytest.approx(64 * 16 ** (1 / 3), rel=1e-15)


def test_quadratic_collapse_removes_the_linear_curvature_bias():
    """Noise-free data of a known scaling form on the default grid: the
    three-point measure returns beta/nu within 2e-3, and closer than the
    linear measure of Houdayer and Hartmann."""
    tc, nu, bn = 4.21394, 0.629, 0.520
    Ls = (32, 48, 64, 96)
    temps = tuple(fss.default_temperatures(workloads.ISING))
    rm = scaling_data(tc, nu, bn, Ls, temps, 3, 0.0, 1)
    U, _, m2, _ = fss.estimates(rm)
    dm2 = 1e-3 * m2
    errs = {}
    for order in (1, 2):
        old = fss.COLLAPSE_ORDER
        fss.COLLAPSE_ORDER = order
        try:
            b, _ = fss.fit_beta_nu(temps, Ls, m2, dm2, tc, nu)
        finally:
            fss.COLLAPSE_ORDER = old
        errs[order] = abs(b - bn)
    assert errs[2] < 2e-3 and errs[2] < errs[1]
