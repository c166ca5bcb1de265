"""Host-side logic of the surrogate's spread calibration and acceptance
gate (no GPU): the least-squares fit recovers a known correction, and the
gate's seed-count threshold and uncertainty guard follow their definitions."""
import numpy as np

from paper_2603_14895_amd import surrogate as S


def test_calibration_recovers_known_correction():
    rng = np.random.default_rng(3)
    q = 600
    beta = rng.uniform(0.01, 0.05, q)
    k = np.round(np.exp(rng.uniform(0, np.log(1000), q))).astype(int)
    true = np.array([0.02, -0.03, 0.01, -0.002, 0.05, -0.01, 0.0, 0.001, -0.0005])
    pred = rng.uniform(1e4, 9e4, q)
    label = pred * np.exp(S.calib_features(beta, k) @ true)
    coef = S.fit_calibration(pred, label, beta, k, min_seeds=1)
    assert np.allclose(coef, true, atol=1e-8)
    assert np.allclose(S.apply_calibration(pred, beta, k, coef), label, rtol=1e-10)


def test_calibration_features_match_definition():
    f = S.calib_features(np.array([0.025]), np.array([4]))[0]
    x, k = 0.5, 4.0
    want = [1, x, x * x, x ** 3, 1 / k, x / k, 1 / k ** 2, np.log(k), x * np.log(k)]
    assert np.allclose(f, want, rtol=0, atol=1e-15)


def test_gate_picks_smallest_reliable_seed_count():
    # errors shrink with the seed count: 8% below 5 seeds, 0.2% from 5 on
    k = np.array([1, 2, 3, 4] * 5 + list(range(5, 45)))
    ref = np.full(k.size, 1e4)
    err = np.where(k < 5, 0.08, 0.002)
    spread = ref * (1 + err)
    unc = np.where(k < 5, 0.05, 0.01)
    g = S.calibrate_gate(spread, unc, ref, k, 0.02, min_seeds_floor=1)
    assert g["min_seeds"] == 5
    assert abs(g["tau"] - 0.01) < 1e-12
    # the floor is respected
    g = S.calibrate_gate(spread, unc, ref, k, 0.02, min_seeds_floor=7)
    assert g["min_seeds"] == 7
    # one large error among the large sets rules every threshold below it out
    spread2 = spread.copy()
    spread2[-1] = ref[-1] * 1.05
    g = S.calibrate_gate(spread2, unc, ref, k, 0.02, min_seeds_floor=1)
    assert g["min_seeds"] > k.max()
    assert g["tau"] < 0
    # the largest calibration error must stay below max_rel_err / safety
    spread3 = spread.copy()
    spread3[-1] = ref[-1] * 1.015
    assert S.calibrate_gate(spread3, unc, ref, k, 0.02, min_seeds_floor=1,
                            safety=1.0)["min_seeds"] == 5
    assert S.calibrate_gate(spread3, unc, ref, k, 0.02, min_seeds_floor=1)["min_seeds"] > k.max()


def test_gate_bounds_uncertainty_and_seed_count_together():
    # near-threshold queries (large member disagreement, 3% error) at every
    # seed count are excluded by the uncertainty bound, not by the seed floor
    k = np.array(list(range(5, 45)) + [6, 15, 25, 35, 44])
    ref = np.full(k.size, 1e4)
    err = np.array([0.002] * 40 + [0.03] * 5)
    unc = np.array([0.01] * 40 + [0.03] * 5)
    g = S.calibrate_gate(ref * (1 + err), unc, ref, k, 0.02, min_seeds_floor=1)
    assert g["min_seeds"] == 5
    assert abs(g["tau"] - 0.01) < 1e-12
    # no pair accepts min_queries queries: everything falls back
    g = S.calibrate_gate(ref * (1 + err), unc, ref, k, 0.02, min_seeds_floor=1, min_queries=41)
    assert g["tau"] < 0 and g["min_seeds"] > k.max()
