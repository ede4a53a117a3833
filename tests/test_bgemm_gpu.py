"""GPU parity of the batched small products (per-class MFMA kernel over a work list, its
HIP-graph replay, and the generic per-instance kernel) against the FP64
oracle.  Bar: |C - C_oracle| <= 1e-12 * (|A||B|)_ij per entry; bit-exact for
identity and small-integer inputs."""
import numpy as np
import pytest

import sj_inputs as gen

from helpers import TOL_F64, dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1904_08555_amd as P
    P.sj_init(0)
    return P


def batch(seed, count, lo=3, hi=16):
    n = gen.batch_sizes(seed, count, lo, hi)
    off = gen.batch_offsets(n)
    A = gen.batch_normal(seed, gen.ARR_A, int(off[-1]))
    B = gen.batch_normal(seed, gen.ARR_B, int(off[-1]))
    return n, off, A, B


def abs_scale(n, off, A, B):
    out = np.empty_like(A)
    for i, s in enumerate(n):
        a = np.abs(A[off[i]:off[i + 1]].reshape(s, s))
        b = np.abs(B[off[i]:off[i + 1]].reshape(s, s))
        out[off[i]:off[i + 1]] = (a @ b).ravel()
    return out


def err(got, ref, scale):
    d = np.abs(got - ref)
    return float(np.max(np.where(scale > 0, d / np.where(scale > 0, scale, 1), np.where(d == 0, 0, np.inf))))


def run_plan(P, n, A_d, B_d, C_d, graph=False, **spec):
    h = P.sj_specialize(P.SJ_BGEMM, **spec)
    plan = P.sj_batch_plan(h, n)
    try:
        if graph:
            P.sj_batch_graph_capture(plan, A_d, B_d, C_d)
            P.sj_batch_graph_launch(plan)
        else:
            P.sj_batch_run(plan, A_d, B_d, C_d)
        torch.cuda.synchronize()
    finally:
        P.sj_plan_destroy(plan)


@pytest.mark.parametrize("spec", [dict(), dict(tile_n=256), dict(unroll=1, block=128), dict(unroll=8, block=512),
                                  dict(unroll=2, block=64, tile_n=1000), dict(order=1), dict(order=3),
                                  dict(order=4, tile_n=1024, block=512), dict(order=3, tile_n=300, block=128),
                                  dict(variant=1), dict(variant=1, unroll=1, block=64, tile_n=256),
                                  dict(variant=1, unroll=4, block=256, tile_n=1024), dict(variant=1, unroll=8, block=64)],
                         ids=["default", "w256", "u1b128", "u8b512", "u2b64", "noprefetch", "prefetch2",
                              "prefetch3-w1024b512", "prefetch2-w300b128",
                              "wave", "wave-u1b64w256", "wave-u4b256w1024", "wave-u8b64"])
@pytest.mark.parametrize("lohi", [(3, 16), (1, 16), (1, 4), (16, 16)], ids=["n3-16", "n1-16", "n1-4", "n16"])
def test_bgemm_small_batches(P, orc, spec, lohi):
    n, off, A, B = batch(7, 777, *lohi)
    ref = orc.bgemm(n, off[:-1], A, B)
    scale = abs_scale(n, off, A, B)
    C_d = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    run_plan(P, n, dev(A), dev(B), C_d, **spec)
    assert err(host(C_d), ref, scale) <= TOL_F64


def test_bgemm_class_mask_and_exact(P, orc):
    n = np.array([5, 3, 5, 16, 3, 5], dtype=np.int32)
    off = gen.batch_offsets(n)
    rng = np.random.default_rng(3)
    B = rng.standard_normal(off[-1])
    A = np.zeros(off[-1])
    for i, s in enumerate(n):
        A[off[i]:off[i + 1]] = np.eye(s).ravel()
    mask = (1 << 3) | (1 << 5) | (1 << 16)
    C_d = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    run_plan(P, n, dev(A), dev(B), C_d, class_mask=mask)
    assert np.array_equal(host(C_d), B)               # identity: C = B bit for bit
    Ai = rng.integers(-9, 10, off[-1]).astype(float)
    Bi = rng.integers(-9, 10, off[-1]).astype(float)
    run_plan(P, n, dev(Ai), dev(Bi), C_d, class_mask=mask)
    assert np.array_equal(host(C_d), orc.bgemm(n, off[:-1], Ai, Bi))
    h = P.sj_specialize(P.SJ_BGEMM, class_mask=mask)
    with pytest.raises(P.SJError) as e:
        P.sj_batch_plan(h, np.array([3, 4], dtype=np.int32))   # class 4 not compiled in
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    with pytest.raises(P.SJError) as e:
        P.sj_batch_plan(h, np.array([3, 17], dtype=np.int32))
    assert e.value.status == P.SJ_ERR_INVALID_ARG


def test_bgemm_empty_plan(P):
    h = P.sj_specialize(P.SJ_BGEMM)
    plan = P.sj_batch_plan(h, np.zeros(0, dtype=np.int32))
    x = torch.zeros(2, dtype=torch.float64, device="cuda")
    y = torch.zeros(2, dtype=torch.float64, device="cuda")
    P.sj_batch_run(plan, x, x, y)
    P.sj_batch_graph_capture(plan, x, x, y)
    P.sj_batch_graph_launch(plan)
    torch.cuda.synchronize()
    P.sj_plan_destroy(plan)


@pytest.mark.parametrize("variant", [0, 1], ids=["workgroup", "wave"])
def test_bgemm_graph_replays(P, orc, variant):
    """The captured graph is replayed several times with eager work and
    synchronizations in between; every replay is checked."""
    n, off, A, B = batch(11, 5000)
    ref = orc.bgemm(n, off[:-1], A, B)
    scale = abs_scale(n, off, A, B)
    A_d, B_d = dev(A), dev(B)
    C_d = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    h = P.sj_specialize(P.SJ_BGEMM, variant=variant)
    plan = P.sj_batch_plan(h, n)
    P.sj_batch_graph_capture(plan, A_d, B_d, C_d)
    for rep in range(4):
        C_d.fill_(float("nan"))
        torch.cuda.synchronize()
        P.sj_batch_graph_launch(plan)
        torch.cuda.synchronize()
        assert err(host(C_d), ref, scale) <= TOL_F64, rep
        _ = (A_d * 2.0).sum().item()   # unrelated eager work between replays
    P.sj_plan_destroy(plan)


def test_bgemm_generic_kernel(P, orc):
    n, off, A, B = batch(13, 3000, 1, 16)
    ref = orc.bgemm(n, off[:-1], A, B)
    scale = abs_scale(n, off, A, B)
    h = P.sj_specialize(P.SJ_BGEMM)
    plan = P.sj_batch_plan(h, n)
    n_dev, off_dev, total = P.sj_batch_plan_arrays(plan)
    assert total == off[-1]
    C_d = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    P.sj_generic_run(P.SJ_BGEMM, [n_dev, off_dev, dev(A), dev(B), C_d], count=len(n))
    torch.cuda.synchronize()
    assert err(host(C_d), ref, scale) <= TOL_F64
    P.sj_plan_destroy(plan)


@pytest.mark.parametrize("variant", [0, 1], ids=["workgroup", "wave"])
def test_bgemm_config_200k(P, orc, variant):
    """200,000 instances, n ~ U{3..16}, A and B ~ N(0,1): every entry checked,
    through the graph replay that the benchmark times."""
    n, off, A, B = batch(0, 200000)
    ref = orc.bgemm(n, off[:-1], A, B)
    C_d = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    run_plan(P, n, dev(A), dev(B), C_d, graph=True, variant=variant)
    got = host(C_d)
    # scale for every entry from |A||B| via the oracle on absolute values
    scale = orc.bgemm(n, off[:-1], np.abs(A), np.abs(B))
    assert err(got, ref, scale) <= TOL_F64


def test_bgemm_alias_rejected(P):
    n = np.array([4, 4], dtype=np.int32)
    h = P.sj_specialize(P.SJ_BGEMM)
    plan = P.sj_batch_plan(h, n)
    buf = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SJError) as e:
        P.sj_batch_run(plan, buf, buf, buf.data_ptr() + 8 * 8)
    assert e.value.status == P.SJ_ERR_ALIAS
    P.sj_plan_destroy(plan)


def test_bgemm_every_tuner_candidate(P, orc):
    """Every tile configuration the batched-product tuner can choose, on a
    mixed batch (sizes 1..16, several windows per workgroup), against the oracle."""
    from paper_1904_08555_amd import tune
    n, off, A, B = batch(11, 3000, 1, 16)
    ref = orc.bgemm(n, off[:-1], A, B)
    scale = abs_scale(n, off, A, B)
    A_d, B_d = dev(A), dev(B)
    C_d = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    for c in tune.bgemm_candidates():
        C_d.fill_(float("nan"))
        run_plan(P, n, A_d, B_d, C_d, **c)
        assert err(host(C_d), ref, scale) <= TOL_F64, c


def test_tune_bgemm_contract(P):
    """tune_bgemm returns the lowest median of the candidates it timed."""
    from paper_1904_08555_amd import tune
    n, off, A, B = batch(12, 2000)
    C_d = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    cands = tune.bgemm_candidates()[:3] + [dict(variant=1, tile_n=100)]      # the last is refused
    r = tune.tune_bgemm(n, dev(A), dev(B), C_d, cands=cands, reps=3)
    assert len(r["results"]) == 3 and [c for c, _ in r["rejected"]] == [cands[3]]
    meds = [m for _, m, _ in r["results"]]
    i = min(range(3), key=lambda k: (meds[k], k))
    assert r["best"] == r["results"][i][0] and r["best_ms"] == meds[i]
