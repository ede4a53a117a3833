"""sj_run_mlp_bwd_noalloc (the allocation-free MLP backward pass, static
device scratch) against sj_run with a caller workspace, through the C ABI:
bit-identical gradients and loss on two calls in a row, the second with
fewer rows; sizes beyond the static scratch are refused."""
import numpy as np
import pytest

from helpers import dev, host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F, H = 30, 64


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1904_08555_amd as P
    P.sj_init(0)
    return P


def one_call(P, rows, seed):
    rng = np.random.default_rng(seed)
    nparam = H * F + H * H + 3 * H + 1
    theta = dev((0.2 * rng.standard_normal(nparam)).astype(np.float32))
    X = dev(rng.standard_normal((rows, F)).astype(np.float32))
    t = dev(rng.standard_normal(rows).astype(np.float32))
    h = P.sj_specialize(P.SJ_MLP_BWD, dtype=P.SJ_F32, rows=rows, inputs=F, width=H)
    g_ref = torch.full((nparam,), float("nan"), dtype=torch.float32, device="cuda")
    l_ref = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    ws = torch.empty(rows * (4 * H + 2), dtype=torch.float32, device="cuda")
    P.sj_run(h, [theta, X, t, g_ref, l_ref, ws])
    g = torch.full((nparam,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    P.sj_run_mlp_bwd_noalloc(h, [theta, X, t, g, loss])
    a, b = host(g), host(g_ref)
    assert np.isfinite(a).all() and np.isfinite(host(loss)).all()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"rows={rows}: gradients differ"
    assert np.array_equal(host(loss).view(np.uint32), host(l_ref).view(np.uint32)), f"rows={rows}: loss differs"


def test_noalloc_matches_workspace_path(P):
    one_call(P, 1000, 1)
    one_call(P, 64, 2)          # a smaller input on the same (shared) scratch


def test_noalloc_refuses_oversize(P):
    rows = (1 << 20) // (4 * H + 2) + 1                  # one row beyond the 4 MiB scratch
    h = P.sj_specialize(P.SJ_MLP_BWD, dtype=P.SJ_F32, rows=rows, inputs=F, width=H)
    nparam = H * F + H * H + 3 * H + 1
    bufs = [torch.zeros(n, dtype=torch.float32, device="cuda") for n in (nparam, rows * F, rows, nparam, 1)]
    with pytest.raises(P.SJError) as e:
        P.sj_run_mlp_bwd_noalloc(h, bufs)
    assert e.value.status == P.SJ_ERR_INVALID_ARG and "static scratch" in e.value.message
    with pytest.raises(P.SJError):                      # not a backward-pass handle
        P.sj_run_mlp_bwd_noalloc(P.sj_specialize(P.SJ_MLP_FWD, dtype=P.SJ_F32, rows=8, inputs=F, width=H),
                                 bufs)
