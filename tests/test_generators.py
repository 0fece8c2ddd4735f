"""The seeded input generators: twins agree bit for bit, recipes hit their targets."""
import numpy as np
import pytest

import coxsim


def test_hash_numpy_and_c_twins_agree():
    _, thr = coxsim.maf_and_thresholds(64, 99)
    cols = np.arange(64)
    a = coxsim.genotype_columns_numpy(777, cols, 99, thr)
    b = coxsim.genotype_columns(777, cols, 99, thr)
    np.testing.assert_array_equal(a, b)
    # a subset of columns regenerates the same values
    sub = np.array([5, 17, 63])
    np.testing.assert_array_equal(coxsim.genotype_columns(777, sub, 99, thr[sub]), a[sub])
    # padding rows beyond n stay zero, FP8 codes are the OCP E4M3 codes of 0/1/2
    f = coxsim.genotype_columns(777, cols, 99, thr, ldx=800, fmt=1)
    np.testing.assert_array_equal(f[:, :777].view(np.uint8), coxsim.FP8_E4M3_CODE[a])
    assert np.all(f[:, 777:] == 0)


def test_splitmix_reference_values():
    # SplitMix64 outputs for state 0 (first three draws of the published
    # generator seeded with 0): mix(k * golden gamma) for k = 1, 2, 3.
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    g = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        got = [int(coxsim.splitmix(np.uint64(k) * g - g)) for k in (1, 2, 3)]
    assert got == want


def test_genotype_frequencies_and_standardisation():
    n = 20000
    maf, thr = coxsim.maf_and_thresholds(40, 3)
    G = coxsim.genotype_columns(n, np.arange(40), 3, thr)
    assert set(np.unique(G)) <= {0, 1, 2}
    # allele frequency within 5 standard errors of maf_j
    freq = G.mean(axis=1) / 2
    se = np.sqrt(maf * (1 - maf) / (2 * n))
    assert np.all(np.abs(freq - maf) < 5 * se)
    c1, c2 = coxsim.genotype_counts(G, n)
    np.testing.assert_array_equal(c1, (G == 1).sum(1))
    np.testing.assert_array_equal(c2, (G == 2).sum(1))
    mu, s = coxsim.standardisation(c1, c2, n)
    assert mu.dtype == np.float32 and s.dtype == np.float32
    Xs = (G - mu[:, None].astype(np.float64)) * s[:, None].astype(np.float64)
    np.testing.assert_allclose(Xs.mean(1), 0, atol=1e-6)
    np.testing.assert_allclose(Xs.var(1), 1, rtol=1e-6)
    mu0, s0 = coxsim.standardisation([0], [0], 10)
    assert s0[0] == 0.0 and mu0[0] == 0.0


@pytest.mark.parametrize("frac", [0.25, 0.3, 0.8])
def test_censoring_fraction(frac):
    rng = np.random.default_rng(0)
    eta = rng.normal(0, 2, size=20000)
    y, d = coxsim.survival_times(eta, frac, rng)
    assert abs((1 - d.mean()) - frac) <= 0.005
    assert np.all(y > 0)


def test_days_give_ties_and_configs():
    d = coxsim.config2(n=5000, p=20)
    assert d.time.min() >= 1 and d.time.max() <= 1000
    assert len(np.unique(d.time)) < 1000
    assert abs((1 - d.event.mean()) - 0.30) <= 0.005
    c0 = coxsim.config0()
    assert c0.G.shape == (2000, 1000) and np.count_nonzero(c0.beta_true) == 10
    lg = coxsim.lambda_grid(2.0, 64)
    assert lg[0] == 2.0 and lg[-1] == pytest.approx(0.02, rel=1e-15) and np.all(np.diff(lg) < 0)
