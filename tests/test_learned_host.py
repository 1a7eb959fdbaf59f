"""Host logic of the learned configuration predictor (no GPU): configuration
keys across workloads whose runnable spaces differ, the masked time matrix,
target distributions, and the regret measures."""
import numpy as np
import pytest

from paper_1910_08498_amd import learned


def rec(keys, ns, default=None):
    return learned.TuneRecord(n=64, slices=100, a=1.9, ns_per_slice=np.array(ns, dtype=float), keys=list(keys),
                              default_key=default)


def test_union_keys_and_time_matrix_mask_missing_configs():
    a = rec([(3, 8, 32, 32, 6), (3, 11, 32, 32, 4)], [2.0, 1.0])
    b = rec([(3, 8, 32, 32, 6), (2, 16, 32, 32, 6)], [3.0, 6.0])
    keys = learned.union_keys([a, b])
    assert keys == [(3, 8, 32, 32, 6), (3, 11, 32, 32, 4), (2, 16, 32, 32, 6)]
    ns = learned.time_matrix([a, b], keys)
    assert ns[0].tolist() == [2.0, 1.0, np.inf]
    assert ns[1].tolist() == [3.0, np.inf, 6.0]


def test_soft_targets_give_no_mass_to_configs_that_do_not_run():
    ns = np.array([[2.0, 1.0, np.inf], [3.0, np.inf, 3.0]])
    y = learned.soft_targets(ns, temperature=0.02)
    assert np.allclose(y.sum(axis=1), 1.0)
    assert y[0, 2] == 0.0 and y[1, 1] == 0.0
    assert y[0, 1] > 0.999                    # the fastest takes almost all mass
    assert np.isclose(y[1, 0], 0.5) and np.isclose(y[1, 2], 0.5)


def test_regret_and_random_search_use_runnable_configs_only():
    ns = np.array([[2.0, 1.0, np.inf, 4.0]])
    assert learned.regret(ns, np.array([1]))[0] == 0.0
    assert learned.regret(ns, np.array([3]))[0] == pytest.approx(3.0)
    # a budget covering every runnable configuration always finds the best
    assert learned.random_search_regret(ns, steps=3, trials=20)[0] == 0.0
    # one random pick: mean over the three runnable configurations of t / t_best - 1
    r1 = learned.random_search_regret(ns, steps=1, trials=3000, seed=1)[0]
    assert r1 == pytest.approx((1.0 + 0.0 + 3.0) / 3, abs=0.1)


def test_cu_mask_spreads_over_blocks_of_the_numbering():
    w = learned.cu_mask_words(64, 256)
    assert len(w) == 8 and sum(bin(x).count("1") for x in w) == 64
    bits = [b for b in range(256) if w[b // 32] >> (b % 32) & 1]
    # 8 per block of 32 (block-major numbering) and 8 per residue mod 8 (round-robin numbering)
    assert np.bincount(np.array(bits) // 32, minlength=8).tolist() == [8] * 8
    assert np.bincount(np.array(bits) % 8, minlength=8).tolist() == [8] * 8
    assert sum(bin(x).count("1") for x in learned.cu_mask_words(256, 256)) == 256
    with pytest.raises(ValueError):
        learned.cu_mask_words(60, 256)


def test_guided_search_and_fallback_policy():
    ns = np.array([[4.0, 1.0, 2.0, np.inf],
                   [1.0, 3.0, 2.0, 5.0]])
    prob = np.array([[0.1, 0.2, 0.6, 0.1],       # ranks config 2 first, config 1 second
                     [0.05, 0.5, 0.05, 0.4]])    # ranks config 1, then 3: never the best
    assert learned.ranked_candidates(prob[0], np.isfinite(ns[0]), 2).tolist() == [2, 1]
    assert learned.ranked_candidates(prob[0], np.isfinite(ns[0]), 9).tolist() == [2, 1, 0]  # runnable only
    g1 = learned.guided_regret(ns, prob, 1)
    g2 = learned.guided_regret(ns, prob, 2)
    assert g1.tolist() == [1.0, 2.0]             # top-1: 2/1 - 1 and 3/1 - 1
    assert g2.tolist() == [0.0, 2.0]             # the second candidate of workload 0 is its best
    assert np.all(learned.guided_regret(ns, prob, 4) == 0.0)
    # confident on workload 0 only (tau = 0.55): workload 1 falls back to a full random search
    reg, steps, fb = learned.policy_regret(ns, prob, 2, 0.55, budget=4, trials=20)
    assert fb.tolist() == [False, True]
    assert steps.tolist() == [2, 4]
    assert reg.tolist() == [0.0, 0.0]


def test_portability_matrix():
    a = rec([(1, 1, 1, 1, 1), (2, 2, 2, 2, 2)], [1.0, 2.0])      # config 0 fastest
    b = rec([(1, 1, 1, 1, 1), (2, 2, 2, 2, 2)], [4.0, 2.0])      # config 1 fastest
    c = rec([(2, 2, 2, 2, 2)], [3.0])                            # config 0 does not run
    m = learned.portability_matrix([a, b, c])
    assert m[0, 0] == 1.0 and m[1, 1] == 1.0 and m[2, 2] == 1.0
    assert m[0, 1] == 0.5                 # a's best on b: 2 / 4
    assert m[1, 0] == 0.5                 # b's best on a: 1 / 2
    assert np.isnan(m[0, 2]) and m[1, 2] == 1.0


def test_guided_search_with_the_default_is_never_worse_than_the_default():
    ns = np.array([[1.0, 1.2, 1.5, 2.0, 1.1], [2.0, 1.0, 3.0, 1.5, 4.0]])
    prob = np.array([[0.1, 0.2, 0.3, 0.35, 0.05], [0.5, 0.1, 0.2, 0.15, 0.05]])
    dflt = np.array([4, 1])
    g3 = learned.guided_regret(ns, prob, 3)
    gd = learned.guided_regret(ns, prob, 3, dflt)
    d = learned.regret(ns, dflt)
    assert np.all(gd <= g3 + 1e-15) and np.all(gd <= d + 1e-15)
    assert gd[1] == 0.0 and g3[1] > 0.0         # the default was the best and not predicted


def test_features_count_slices_per_call():
    f = learned.features(128, 50000, 1.9, 0.5)
    assert f[0] == 7.0 and f[1] == pytest.approx(np.log2(1500)) and f[2] == 1.9 and f[3] == 0.5
    assert learned.features(128, 1000, 1.9, 1.0)[1] == pytest.approx(np.log2(1000))


def test_tune_record_round_trip(tmp_path):
    from paper_1910_08498_amd.learned import TuneRecord
    r = TuneRecord(n=96, slices=1234, a=1.7, ns_per_slice=np.array([3.0, 2.5, 4.0]),
                   keys=[(3, 11, 64, 32, 4, 1, 0), (3, 8, 32, 16, 6, 1, 3), (2, 16, 32, 16, 6, 1, 2)],
                   default_key=(3, 11, 64, 32, 4, 1, 0), cus=128, cus_total=256)
    r.save(str(tmp_path / "r.npz"))
    q = TuneRecord.load(str(tmp_path / "r.npz"))
    assert (q.n, q.slices, q.a, q.cus, q.cus_total) == (96, 1234, 1.7, 128, 256)
    assert q.keys == r.keys and q.default_key == r.default_key
    assert np.array_equal(q.ns_per_slice, r.ns_per_slice)
    assert np.allclose(q.features(), r.features())


def test_tune_record_keys_without_traversal_load_with_the_default(tmp_path):
    """Records written before the traversal knob hold six-value keys; they
    load with traversal 0, the only value those timings covered."""
    from paper_1910_08498_amd.learned import TuneRecord
    r = TuneRecord(n=64, slices=500, a=1.9, ns_per_slice=np.array([1.0, 2.0]),
                   keys=[(3, 11, 64, 32, 4, 1), (3, 8, 32, 16, 6, 1)], default_key=(3, 11, 64, 32, 4, 1),
                   cus=256, cus_total=256)
    r.save(str(tmp_path / "old.npz"))
    q = TuneRecord.load(str(tmp_path / "old.npz"))
    assert q.keys == [(3, 11, 64, 32, 4, 1, 0), (3, 8, 32, 16, 6, 1, 0)]
    assert q.default_key == (3, 11, 64, 32, 4, 1, 0)
