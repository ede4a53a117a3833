"""GPU parity of the tensor-product mass operator (partial assembly, sum
factorization) against the FP64 CPU oracle (plain quadrature sums), through
the C ABI.  Bar: componentwise |gpu - oracle| <= 1e-12 * (|B|^T |D| |B| |x|)
(helpers.TOL_F64); bit-exact where every partial sum is exact."""
import numpy as np
import pytest

from helpers import TOL_F64, componentwise_err, dev, host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1904_08555_amd as P
    P.sj_init(0)
    return P


def inputs(seed, dim, D1D, Q1D, NE):
    rng = np.random.default_rng(seed)
    B1 = rng.uniform(-1, 1, (Q1D, D1D))
    Dq = rng.uniform(0.1, 2.0, NE * Q1D ** dim)
    X = rng.uniform(-1, 1, NE * D1D ** dim)
    return B1, Dq, X


def run(P, dim, D1D, Q1D, NE, B1, Dq, X, **tile):
    Y = torch.empty(NE * D1D ** dim, dtype=torch.float64, device="cuda")
    h = P.sj_specialize(P.SJ_MASS, D=D1D, NM=Q1D, inputs=dim, count=NE, **tile)
    P.sj_run(h, [dev(B1.ravel()), dev(Dq), dev(X), Y])
    return host(Y)


@pytest.mark.parametrize("shape", [(1, 5, 7, 33), (2, 4, 6, 101), (2, 3, 3, 7), (3, 2, 3, 50), (3, 4, 6, 37),
                                   (3, 5, 4, 9), (2, 8, 12, 19), (3, 1, 1, 3), (1, 1, 2, 200), (3, 8, 12, 5)],
                         ids=lambda s: "dim%dD%dQ%dNE%d" % s)
@pytest.mark.parametrize("tile", [dict(), dict(tile_n=1, block=64), dict(tile_n=3, block=256),
                                  dict(order=1), dict(order=2), dict(order=2, tile_n=3, block=256),
                                  dict(order=1, tile_n=2, block=128)],
                         ids=["default", "ew1", "ew3", "staged", "pipelined", "pipelined-ew3", "staged-ew2"])
def test_mass_parity(P, orc, shape, tile):
    dim, D1D, Q1D, NE = shape
    B1, Dq, X = inputs(61, dim, D1D, Q1D, NE)
    try:
        got = run(P, dim, D1D, Q1D, NE, B1, Dq, X, **tile)
    except P.SJError as e:   # an explicit tile whose LDS tiles do not fit is refused, not run
        assert tile and e.status == P.SJ_ERR_UNSUPPORTED, e
        return
    ref = orc.mass(dim, D1D, Q1D, B1, Dq, X)
    scale = orc.mass(dim, D1D, Q1D, B1, Dq, X, absolute=True)
    assert componentwise_err(got, ref, scale) <= TOL_F64


def test_mass_identity_and_integer_exact(P, orc):
    dim, D1D, NE = 3, 4, 70
    rng = np.random.default_rng(62)
    Dq = rng.uniform(-2, 2, NE * D1D ** dim)
    X = rng.uniform(-2, 2, NE * D1D ** dim)
    assert np.array_equal(run(P, dim, D1D, D1D, NE, np.eye(D1D), Dq, X), Dq * X)
    Q1D = 5
    B1 = rng.integers(-3, 4, (Q1D, D1D)).astype(np.float64)
    Dq = rng.integers(1, 5, NE * Q1D ** dim).astype(np.float64)
    X = rng.integers(-4, 5, NE * D1D ** dim).astype(np.float64)
    assert np.array_equal(run(P, dim, D1D, Q1D, NE, B1, Dq, X), orc.mass(dim, D1D, Q1D, B1, Dq, X))


def test_mass_checks(P):
    h = P.sj_specialize(P.SJ_MASS, D=2, NM=3, inputs=2, count=4)
    x = torch.zeros(4096, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SJError) as e:
        P.sj_run(h, [x, x, x])
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    with pytest.raises(P.SJError) as e:   # Y overlaps X
        P.sj_run(h, [x, x.data_ptr() + 1024, x.data_ptr() + 2048, x.data_ptr() + 2048])
    assert e.value.status == P.SJ_ERR_ALIAS


def test_mass_full_size_sampled(P, orc):
    """NE = 500,000 hexahedra, D1D = 4, Q1D = 6 (the benchmark's size): 2000
    sampled elements against the oracle."""
    dim, D1D, Q1D, NE = 3, 4, 6, 500000
    rng = np.random.default_rng(63)
    B1 = rng.uniform(-1, 1, (Q1D, D1D))
    Dq_d = torch.rand(NE * Q1D ** dim, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    X_d = torch.rand(NE * D1D ** dim, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(2))
    Y_d = torch.empty_like(X_d)
    h = P.sj_specialize(P.SJ_MASS, D=D1D, NM=Q1D, inputs=dim, count=NE)
    P.sj_run(h, [dev(B1.ravel()), Dq_d, X_d, Y_d])
    es = np.sort(rng.choice(NE, 2000, replace=False))
    es[-1] = NE - 1
    nd, nq = D1D ** dim, Q1D ** dim
    Xs = host(X_d).reshape(NE, nd)[es]
    Ds = host(Dq_d).reshape(NE, nq)[es]
    ref = orc.mass(dim, D1D, Q1D, B1, Ds.ravel(), Xs.ravel())
    scale = orc.mass(dim, D1D, Q1D, B1, Ds.ravel(), Xs.ravel(), absolute=True)
    got = host(Y_d).reshape(NE, nd)[es].ravel()
    assert componentwise_err(got, ref, scale) <= TOL_F64
    del Dq_d, X_d, Y_d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("shape", [(1, 32, 32, 37), (2, 32, 32, 5), (2, 32, 1, 9), (2, 1, 32, 9), (3, 18, 18, 2),
                                   (3, 16, 18, 3)],
                         ids=lambda s: "dim%dD%dQ%dNE%d" % s)
def test_mass_parity_range_edges(P, orc, shape):
    """The largest sizes the specializer accepts: D1D = Q1D = 32 for dim 1 and 2,
    and D1D = Q1D = 18 for dim 3 (one element's LDS tiles fill 160 KiB at 18)."""
    dim, D1D, Q1D, NE = shape
    B1, Dq, X = inputs(64, dim, D1D, Q1D, NE)
    got = run(P, dim, D1D, Q1D, NE, B1, Dq, X)
    ref = orc.mass(dim, D1D, Q1D, B1, Dq, X)
    scale = orc.mass(dim, D1D, Q1D, B1, Dq, X, absolute=True)
    assert componentwise_err(got, ref, scale) <= TOL_F64
    if dim == 3:
        return   # the pipelined form's registers spill at these sizes; only the staged form is the default
    got = run(P, dim, D1D, Q1D, NE, B1, Dq, X, order=2)
    ref = orc.mass(dim, D1D, Q1D, B1, Dq, X)
    scale = orc.mass(dim, D1D, Q1D, B1, Dq, X, absolute=True)
    assert componentwise_err(got, ref, scale) <= TOL_F64
