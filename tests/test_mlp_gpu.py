"""GPU parity of the cost-model MLP kernels (FP32) against the FP64 oracle,
and a small end-to-end check of the picker.  Bars: forward and loss within
1e-5 relative, gradient within 1e-4 normwise relative, Adam within 1e-6."""
import numpy as np
import pytest

from helpers import dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1904_08555_amd as P
    P.sj_init(0)
    return P


def setup(F, H, R, seed):
    import oracle
    rng = np.random.default_rng(seed)
    theta = (rng.standard_normal(oracle.mlp_nparams(F, H)) * 0.3).astype(np.float32)
    X = rng.standard_normal((R, F)).astype(np.float32)
    t = rng.standard_normal(R).astype(np.float32)
    return theta, X, t


@pytest.mark.parametrize("F,H,R", [(24, 64, 128), (24, 64, 1000), (5, 7, 3), (1, 1, 1), (17, 33, 70)])
def test_mlp_forward_and_gradient(P, orc, F, H, R):
    theta, X, t = setup(F, H, R, F + H + R)
    hf = P.sj_specialize(P.SJ_MLP_FWD, dtype=P.SJ_F32, rows=R, inputs=F, width=H)
    hb = P.sj_specialize(P.SJ_MLP_BWD, dtype=P.SJ_F32, rows=R, inputs=F, width=H)
    th_d, X_d, t_d = dev(theta), dev(X), dev(t)
    y_d = torch.empty(R, dtype=torch.float32, device="cuda")
    P.sj_run(hf, [th_d, X_d, y_d])
    y_ref = orc.mlp_forward(F, H, theta.astype(np.float64), X.astype(np.float64))
    y = host(y_d).astype(np.float64)
    assert np.abs(y - y_ref).max() <= 1e-5 * max(1.0, np.abs(y_ref).max())
    g_d = torch.empty(theta.size, dtype=torch.float32, device="cuda")
    loss_d = torch.empty(1, dtype=torch.float32, device="cuda")
    ws = torch.empty(R * (4 * H + 2), dtype=torch.float32, device="cuda")
    P.sj_run(hb, [th_d, X_d, t_d, g_d, loss_d, ws])
    loss_ref, g_ref = orc.mlp_loss_grad(F, H, theta.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    g = host(g_d).astype(np.float64)
    assert abs(float(host(loss_d)[0]) - loss_ref) <= 1e-5 * max(1.0, loss_ref)
    assert np.linalg.norm(g - g_ref) <= 1e-4 * max(np.linalg.norm(g_ref), 1e-30)


def test_adam_matches_oracle(P, orc):
    n = 5000
    rng = np.random.default_rng(1)
    p = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    h = P.sj_specialize(P.SJ_ADAM, dtype=P.SJ_F32, rows=n)
    p_d, m_d, v_d = dev(p), dev(m), dev(v)
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        P.sj_run_adam(h, [p_d, dev(g), m_d, v_d], step, lr=1e-2)
        orc.adam(pr, g.astype(np.float64), mr, vr, step, lr=1e-2)
    assert np.abs(host(p_d) - pr).max() <= 1e-6 * max(1.0, np.abs(pr).max())
    with pytest.raises(P.SJError):
        P.sj_run_adam(h, [p_d, p_d, m_d, v_d], 1)   # g aliases p


def test_mlp_training_reduces_loss(P):
    from paper_1904_08555_amd.picker import MLP
    rng = np.random.default_rng(0)
    X = rng.standard_normal((1024, 24)).astype(np.float32)
    y = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    mlp = MLP(nfeat=24, seed=0)
    with pytest.raises(ValueError):
        MLP(seed=0, nfeat=30).fit(X, y, epochs=1)    # rows of the wrong width are refused on the host
    losses = mlp.fit(X, y, epochs=60, batch=128, lr=3e-3)
    assert losses[-1] < 0.25 * losses[0]
    pred = mlp.predict(X)
    assert np.mean((pred - y) ** 2) < 0.3 * np.var(y)


@pytest.mark.timeout(900)
def test_picker_gain_small(P):
    """A reduced picker experiment (zones up to 24^3, three nestings, 640
    training timings, 16 held-out shapes each timed over the exhaustive
    tuner's whole candidate set).  What the trained network gains over the
    method without it: against the exhaustive tuner, it compiles at most KMAX
    candidates (a quarter of the set or less) instead of all of them, at a
    small regret; against the untuned
    default, its choice is faster; against a choice made without a model (a
    random candidate), its regret is a fraction."""
    from paper_1904_08555_amd import picker
    data = picker.collect(n_train_shapes=80, per_shape=8, n_eval=16, seed=3, workers=12, max_k=24,
                          layouts=("DGZ", "GDZ", "ZGD"), log=lambda m: print(m, flush=True))
    res, _, _ = picker.evaluate(data, seed=3, epochs=150, log=lambda m: print(m, flush=True))
    print(res)
    assert res["eval_shapes"] >= 14
    assert res["compiles_mean"] <= picker.KMAX and res["compiles_mean"] <= 0.25 * res["candidates_mean"]
    assert res["shortlist_regret_mean"] <= res["regret_mean"]
    assert res["shortlist_regret_mean"] <= 0.15
    assert res["regret_mean"] < 0.5 * res["random_choice_regret_mean"]
    assert res["shortlist_speedup_vs_default_geomean"] > 1.0


def test_pretrained_picker(P, orc):
    """The ensemble shipped with the package: its predictions are the FP64
    oracle's forward pass of the shipped weights over the standardized features
    (within the forward bar), and its pick and shortlist come from the shape's
    candidate set."""
    from paper_1904_08555_amd import picker
    pk = picker.Picker.pretrained()
    assert len(pk.mlps) == 5
    d = picker._load_weights(picker.PRETRAINED)
    rng = np.random.default_rng(11)
    for s in picker.draw_shapes(rng, 3):
        cands = picker.candidates(s)
        F = pk._norm(np.stack([picker.features(s, c) for c in cands]))
        got = pk.predict_members(s, cands)
        for k, th in enumerate(d["thetas"]):
            ref = orc.mlp_forward(picker.NFEAT, picker.WIDTH, np.asarray(th, dtype=np.float64),
                                  F.astype(np.float32).astype(np.float64)) * pk.tsd
            assert np.abs(got[k] - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max()) * max(1.0, pk.tsd)
        choice, _ = pk.pick(s, cands)
        assert choice in cands
        short, _ = pk.shortlist(s, cands)
        assert 1 <= len(short) <= picker.KMAX and all(0 <= j < len(cands) for j in short)
