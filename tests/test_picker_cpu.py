"""The learned picker's host logic: its candidate set is the exhaustive
tuner's, its features describe the resolved specialization, and its
shortlist rule (the fallback to timing) follows the ensemble's spread.  The
networks themselves run on the GPU (tests/test_mlp_gpu.py)."""
import json

import numpy as np

from paper_1904_08555_amd import picker, sj, tune


def test_candidate_set_is_the_tuners():
    rng = np.random.default_rng(5)
    for s in picker.draw_shapes(rng, 12):
        got = picker.candidates(s)
        want = []
        for lay in sj.LAYOUTS:
            for c in tune.candidates(sj.SJ_LTIMES, lay, s["Z"], s["G"], s["D"], s["NM"], s["dtype"]):
                try:
                    sj.sj_resolve(sj.SJ_LTIMES, **picker.spec_of(s, dict(layout=lay, **c)))
                except sj.SJError:
                    continue
                want.append(dict(layout=lay, **c))
        assert [json.dumps(c, sort_keys=True) for c in got] == [json.dumps(c, sort_keys=True) for c in want]
        assert got


def test_features_follow_the_resolved_spec():
    s = dict(Z=32768, G=32, D=96, NM=16, dtype=sj.SJ_F64)
    # the default request and the explicit spelling of what it resolves to give one feature vector
    r = sj.sj_resolve(sj.SJ_LTIMES, **picker.spec_of(s, dict(layout="DGZ")))
    explicit = dict(layout="DGZ", variant=r["variant"], tile_n=r["tile_n"], unroll=r["unroll"], block=r["block"],
                    order=r["order"], flags=r["flags"] & ~sj.SJ_FLAG_INDEX64)
    assert np.array_equal(picker.features(s, dict(layout="DGZ")), picker.features(s, explicit))
    cs = picker.candidates(s)
    F = np.stack([picker.features(s, c) for c in cs])
    assert F.shape == (len(cs), picker.NFEAT) and np.isfinite(F).all()
    # distinct specializations are told apart
    assert len({tuple(row) for row in F}) == len(cs)


class _FakeEnsemble(picker.Picker):
    def __init__(self, preds):
        self.preds = np.asarray(preds, dtype=np.float64)

    def predict_members(self, shape, cands):
        return self.preds


def test_shortlist_follows_the_spread():
    # member predictions for 5 candidates; means 0.0, 0.05, 1.0, 0.02, 0.5
    confident = _FakeEnsemble([[0.0, 0.05, 1.0, 0.02, 0.5]] * 3)        # no spread: one compile
    idx, mu = confident.shortlist({}, [None] * 5)
    assert idx == [0] and np.allclose(mu, [0.0, 0.05, 1.0, 0.02, 0.5])
    unsure = _FakeEnsemble([[0.0, 0.10, 1.0, 0.00, 0.5],
                            [0.02, 0.00, 1.0, 0.04, 0.5],
                            [-0.02, 0.05, 1.0, 0.02, 0.5]])
    idx, _ = unsure.shortlist({}, [None] * 5)
    # 0 first, then 3 and 1 (in predicted order) are within the spread; 4 and 2 are not
    assert idx == [0, 3, 1]
    idx, _ = unsure.shortlist({}, [None] * 5, kmax=2)
    assert idx == [0, 3]
    # ties in the mean go to the lowest candidate index
    tie = _FakeEnsemble([[0.3, 0.1, 0.1]])
    assert tie.shortlist({}, [None] * 3)[0] == [1]


def test_held_out_shapes_do_not_depend_on_extra_training_shapes():
    key = lambda shapes: [json.dumps(s, sort_keys=True) for s in shapes]   # noqa: E731
    tr0, ev0 = picker.experiment_shapes(250, 200, seed=0)
    tr1, ev1 = picker.experiment_shapes(250, 200, seed=0, extra_train_shapes=500)
    assert key(ev0) == key(ev1) and len(ev1) == 200
    assert key(tr1[:250]) == key(tr0) and len(tr1) == 750
    # every drawn shape respects the zone limit, and no training shape is a held-out one
    assert all(round(s["Z"] ** (1 / 3)) <= 64 for s in tr1 + ev1)
    assert not set(key(tr1)) & set(key(ev1))


def test_pretrained_weights_ship_with_the_package():
    """The shipped ensemble loads without unpickling and matches the network the
    module builds; a JSON round trip through the converter keeps every value."""
    d = picker._load_weights(picker.PRETRAINED)
    P = picker.WIDTH * picker.NFEAT + picker.WIDTH * picker.WIDTH + 3 * picker.WIDTH + 1
    assert np.asarray(d["thetas"]).shape == (5, P) and np.isfinite(d["thetas"]).all()
    assert np.all(np.asarray(d["sd"]) > 0) and float(d["tsd"]) > 0


def test_weights_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    P = picker.WIDTH * picker.NFEAT + picker.WIDTH * picker.WIDTH + 3 * picker.WIDTH + 1
    d = dict(thetas=rng.standard_normal((2, P)).astype(np.float32).tolist(), mu=rng.standard_normal(picker.NFEAT).tolist(),
             sd=(1 + rng.random(picker.NFEAT)).tolist(), tsd=0.7, nfeat=picker.NFEAT, width=picker.WIDTH)
    (tmp_path / "w.json").write_text(json.dumps(d))
    picker.weights_to_npz(str(tmp_path / "w.json"), str(tmp_path / "w.npz"))
    back = picker._load_weights(str(tmp_path / "w.npz"))
    assert np.array_equal(np.asarray(back["thetas"]), np.asarray(d["thetas"], dtype=np.float32))
    assert np.array_equal(back["mu"], d["mu"]) and np.array_equal(back["sd"], d["sd"]) and float(back["tsd"]) == 0.7
    d["width"] = 32
    (tmp_path / "bad.json").write_text(json.dumps(d))
    import pytest
    with pytest.raises(ValueError):
        picker._load_weights(str(tmp_path / "bad.json"))


def test_evaluate_scores_regret_by_its_definition():
    """evaluate() against hand-computed regrets: r = t(choice) / min t - 1 per shape,
    then the mean; the shortlist keeps its fastest member; the random choice is the
    mean regret over the whole set; the default and the speedup over it likewise."""
    class Fixed(picker.Picker):
        def __init__(self, table):
            self.table = table

        def predict_members(self, shape, cands):
            return np.asarray(self.table[shape["k"]], dtype=np.float64)

    rows = [
        # shape 0: the model is sure of candidate 0 (2.0 ms), the best is candidate 1 (1.0 ms)
        dict(shape=dict(k=0), times=[("a", 2.0), ("b", 1.0), ("c", 4.0)], default_ms=3.0),
        # shape 1: the model cannot separate candidates 1 and 2; the shortlist times both
        dict(shape=dict(k=1), times=[("a", 5.0), ("b", 3.0), ("c", 2.5)], default_ms=2.5),
    ]
    table = {0: [[0.0, 1.0, 2.0]] * 3,
             1: [[1.0, 0.0, 0.01], [1.0, 0.02, 0.0], [1.0, 0.01, 0.02]]}
    res, _, out = picker.evaluate(dict(eval=rows), picker=Fixed(table), log=lambda m: None)
    pick = [2.0 / 1.0 - 1, 3.0 / 2.5 - 1]            # shape 1 picks b (mean 0.01 < 0.01 + ...)
    short = [2.0 / 1.0 - 1, 0.0]                       # shape 1's shortlist holds c
    rand = [np.mean([1.0, 0.0, 3.0]), np.mean([1.0, 0.2, 0.0])]
    dflt = [3.0 / 1.0 - 1, 0.0]
    assert [r["pick"] for r in out] == ["a", "b"] and [r["t_best"] for r in out] == [1.0, 2.5]
    assert res["eval_shapes"] == 2 and res["compiles_mean"] == 1.5
    assert np.isclose(res["regret_mean"], np.mean(pick), atol=1e-4)
    assert np.isclose(res["shortlist_regret_mean"], np.mean(short), atol=1e-4)
    assert np.isclose(res["random_choice_regret_mean"], np.mean(rand), atol=1e-4)
    assert np.isclose(res["default_regret_mean"], np.mean(dflt), atol=1e-4)
    assert np.isclose(res["speedup_vs_default_geomean"], np.sqrt(3.0 / 2.0 * 2.5 / 3.0), atol=1e-4)
    assert res["within_10pct"] == 0.0 and res["shortlist_within_10pct"] == 0.5
