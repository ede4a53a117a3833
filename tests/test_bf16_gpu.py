"""GPU checks of the split-BF16 LTimes (MFMA, FP32 accumulation) against the
FP64 oracle.  psi is FP32 with 24 random bits (exactly representable), L is
FP64.  Bounds, with u_b = 2^-8 (bfloat16) and gamma_s(n) = n u_s / (1 - n u_s),
u_s = 2^-24 (FP32), relative to s = sum_d |L||psi|:
  plain (hi*hi):              |phi - exact| <= (2 u_b + u_b^2 + gamma_s(D + 1)) s
  compensated (hi*hi+hi*lo+lo*hi): |phi - exact| <= (3 u_b^2 + gamma_s(3D + 1)) s
and, tighter, against the oracle's FP64 evaluation of the same split terms:
  |phi - emulated| <= gamma_s(3D + 1) * s * (1 + 2 u_b)
"""
import numpy as np
import pytest

import sj_inputs as gen
from sj_inputs import device as gdev

from helpers import componentwise_err, dev, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

UB = 2.0 ** -8
US = 2.0 ** -24


def gs(n):
    return n * US / (1 - n * US)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1904_08555_amd as P
    P.sj_init(0)
    return P


def bf16_inputs(seed, layout, Z, G, D, NM):
    psi = gen.to_layout(gen.psi_logical(seed, D, G, Z, bits24=True), layout).ravel()
    L = gen.matrix_sym(seed, gen.ARR_L, NM, D)
    return L, psi


def run_bf16(P, dtype, layout, Z, G, D, NM, L_d, psi_d, **tile):
    phi_d = torch.empty(NM * G * Z, dtype=torch.float32, device="cuda")
    h = P.sj_specialize(P.SJ_LTIMES, layout=layout, Z=Z, G=G, D=D, NM=NM, dtype=dtype, **tile)
    P.sj_run(h, [L_d, psi_d, phi_d])
    return phi_d


SHAPES = [(37, 5, 11, 6), (300, 3, 48, 16), (64, 2, 128, 64), (1, 33, 7, 40), (96, 4, 96, 16), (5, 7, 250, 3),
          (37, 5, 12, 6), (1, 33, 20, 40), (5, 7, 252, 3), (33, 1, 16, 33), (3, 3, 4, 1)]


@pytest.mark.parametrize("layout", ["DGZ", "DZG", "GDZ", "ZDG", "GZD", "ZGD"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "Z%dG%dD%dNM%d" % s)
def test_bf16_bounds(P, orc, layout, shape):
    Z, G, D, NM = shape
    if {"DGZ": G * Z, "DZG": G * Z, "GDZ": Z, "ZDG": G}.get(layout, 1) == 1 and D % 4 != 0:
        with pytest.raises(P.SJError) as e:
            P.sj_specialize(P.SJ_LTIMES, layout=layout, Z=Z, G=G, D=D, NM=NM, dtype=P.SJ_BF16)
        assert e.value.status == P.SJ_ERR_UNSUPPORTED   # rows of D values read as 16-byte pieces: D % 4 == 0
        return
    L, psi = bf16_inputs(2, layout, Z, G, D, NM)
    exact = orc.ltimes(layout, Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)
    L_d, psi_d = dev(L), dev(psi.astype(np.float32))
    plain = host(run_bf16(P, P.SJ_BF16, layout, Z, G, D, NM, L_d, psi_d)).astype(np.float64)
    comp = host(run_bf16(P, P.SJ_BF16X3, layout, Z, G, D, NM, L_d, psi_d)).astype(np.float64)
    e_plain = componentwise_err(plain, exact, scale)
    e_comp = componentwise_err(comp, exact, scale)
    assert e_plain <= 2 * UB + UB * UB + gs(D + 1)
    assert e_comp <= 3 * UB * UB + gs(3 * D + 1)
    emul0 = orc.ltimes_bf16_emul(0, layout, Z, G, D, NM, L, psi)
    emul1 = orc.ltimes_bf16_emul(1, layout, Z, G, D, NM, L, psi)
    assert componentwise_err(plain, emul0, scale) <= gs(D + 1) * (1 + 2 * UB)
    assert componentwise_err(comp, emul1, scale) <= gs(3 * D + 1) * (1 + 2 * UB)


def test_bf16_exact_inputs(P, orc):
    """Inputs already exact in bfloat16: lo parts vanish, both modes equal the
    FP64 result up to FP32 accumulation; small integers make it exact."""
    Z, G, D, NM = 64, 3, 32, 8
    rng = np.random.default_rng(4)
    Li = rng.integers(-4, 5, (NM, D)).astype(float)
    pi = rng.integers(0, 8, D * G * Z).astype(float)
    ref = orc.ltimes("DGZ", Z, G, D, NM, Li, pi)
    for dt in (P.SJ_BF16, P.SJ_BF16X3):
        got = host(run_bf16(P, dt, "DGZ", Z, G, D, NM, dev(Li), dev(pi.astype(np.float32))))
        assert np.array_equal(got.astype(np.float64), ref)


def test_bf16_block_sizes(P, orc):
    Z, G, D, NM = 200, 2, 40, 20
    L, psi = bf16_inputs(3, "GDZ", Z, G, D, NM)
    exact = orc.ltimes("GDZ", Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale("GDZ", Z, G, D, NM, L, psi)
    for block in (64, 128, 512, 1024):
        got = host(run_bf16(P, P.SJ_BF16X3, "GDZ", Z, G, D, NM, dev(L), dev(psi.astype(np.float32)), block=block))
        assert componentwise_err(got, exact, scale) <= 3 * UB * UB + gs(3 * D + 1)


def test_bf16_d_innermost_limits(P):
    """With D innermost the rows are read in 16-byte pieces: D % 4 != 0 is
    refused, and the row form takes no other tile than one 32-row tile per wave."""
    with pytest.raises(P.SJError) as e:
        P.sj_specialize(P.SJ_LTIMES, layout="GZD", Z=4, G=2, D=10, NM=4, dtype=P.SJ_BF16)
    assert e.value.status == P.SJ_ERR_UNSUPPORTED
    with pytest.raises(P.SJError) as e:
        P.sj_specialize(P.SJ_LTIMES, layout="ZGD", Z=4, G=2, D=8, NM=4, dtype=P.SJ_BF16, tile_n=4)
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    h = P.sj_specialize(P.SJ_LTIMES, layout="ZGD", Z=4, G=2, D=8, NM=4, dtype=P.SJ_BF16X3)
    assert P.sj_handle_info(h)["kernel_name"].startswith("sj_ltimes_bf16x3_rows")


@pytest.mark.parametrize("layout", ["GZD", "ZGD"])
def test_bf16_rows_large_sampled(P, orc, layout):
    """D innermost at Z=262144 G=64 D=128 NM=64 (psi 8.6 GB FP32): both modes,
    1024 sampled columns against the oracle and the stated bounds."""
    from helpers import gather_columns, sample_columns
    Z, G, D, NM = 262144, 64, 128, 64
    li = gen.LAYOUTS.index(layout)
    psi_d = torch.empty(D * G * Z, dtype=torch.float32, device="cuda")
    gdev.fill(psi_d, 0, gen.ARR_PSI, gdev.DIST_U01_24, li, (D, G, Z))
    L = gen.matrix_sym(0, gen.ARR_L, NM, D)
    g, z = sample_columns(7 + li, G, Z, 1024)
    cols = gen.psi_columns(0, D, G, Z, g, z, bits24=True)
    exact = orc.ltimes("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    scale = orc.ltimes_absscale("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    errs = {}
    for dt, bound in ((P.SJ_BF16, 2 * UB + UB * UB + gs(D + 1)), (P.SJ_BF16X3, 3 * UB * UB + gs(3 * D + 1))):
        phi_d = run_bf16(P, dt, layout, Z, G, D, NM, dev(L), psi_d)
        got = gather_columns(phi_d, layout, NM, G, Z, g, z).astype(np.float64)
        errs[dt] = componentwise_err(got, exact, scale)
        assert errs[dt] <= bound
        del phi_d
        torch.cuda.empty_cache()
    print(f"{layout}: observed max componentwise error plain {errs[P.SJ_BF16]:.3e}, compensated {errs[P.SJ_BF16X3]:.3e}")
    assert errs[P.SJ_BF16X3] < errs[P.SJ_BF16] / 50
    del psi_d
    torch.cuda.empty_cache()


def test_bf16_large_config_sampled(P, orc):
    """Z=262144 G=64 D=128 NM=64 (psi has 2^31 elements: 64-bit indexing), DGZ,
    both modes in both the wide (default) and narrow forms; sampled columns
    against the oracle.  Reports the observed maximum errors."""
    Z, G, D, NM = 262144, 64, 128, 64
    psi_d = torch.empty(D * G * Z, dtype=torch.float32, device="cuda")
    gdev.fill(psi_d, 0, gen.ARR_PSI, gdev.DIST_U01_24, 0, (D, G, Z))
    L = gen.matrix_sym(0, gen.ARR_L, NM, D)
    L_d = dev(L)
    rng = np.random.default_rng(5)
    g = rng.integers(0, G, 1024)
    z = rng.integers(0, Z, 1024)
    g[:2], z[:2] = [0, G - 1], [0, Z - 1]
    cols = gen.psi_columns(0, D, G, Z, g, z, bits24=True)
    exact = orc.ltimes("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    scale = orc.ltimes_absscale("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    flat = (g.astype(np.int64) * Z + z)
    errs = {}
    idx = torch.from_numpy(np.arange(NM)[:, None] * (G * Z) + flat[None, :]).cuda().reshape(-1)
    for cols_per_lane in (0, 1):
        for dt, bound in ((P.SJ_BF16, 2 * UB + UB * UB + gs(D + 1)), (P.SJ_BF16X3, 3 * UB * UB + gs(3 * D + 1))):
            phi_d = run_bf16(P, dt, "DGZ", Z, G, D, NM, L_d, psi_d, tile_n=cols_per_lane)
            got = host(phi_d[idx]).astype(np.float64).reshape(NM, -1)
            errs[(dt, cols_per_lane)] = componentwise_err(got, exact, scale)
            assert errs[(dt, cols_per_lane)] <= bound
            del phi_d
            torch.cuda.empty_cache()
    print("observed max componentwise error: plain %.3e / %.3e, compensated %.3e / %.3e (wide / narrow)"
          % (errs[(P.SJ_BF16, 0)], errs[(P.SJ_BF16, 1)], errs[(P.SJ_BF16X3, 0)], errs[(P.SJ_BF16X3, 1)]))
    for c in (0, 1):
        assert errs[(P.SJ_BF16X3, c)] < errs[(P.SJ_BF16, c)] / 50
    del psi_d
    torch.cuda.empty_cache()


def test_fp64_large_config_sampled(P, orc):
    """The FP64 paths the benchmark times beside BF16 at Z=262144 G=64 D=128
    NM=64 (DGZ, psi 17 GB): vector FMAs (DIRECT) and the FP64 matrix-core
    column kernel, on the same 24-bit values; sampled columns against the
    oracle at the FP64 bar."""
    from helpers import TOL_F64
    Z, G, D, NM = 262144, 64, 128, 64
    psi_d = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
    gdev.fill(psi_d, 0, gen.ARR_PSI, gdev.DIST_U01_24, 0, (D, G, Z))
    L = gen.matrix_sym(0, gen.ARR_L, NM, D)
    L_d = dev(L)
    rng = np.random.default_rng(6)
    g = rng.integers(0, G, 1024)
    z = rng.integers(0, Z, 1024)
    g[:2], z[:2] = [0, G - 1], [0, Z - 1]
    cols = gen.psi_columns(0, D, G, Z, g, z, bits24=True)
    exact = orc.ltimes("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    scale = orc.ltimes_absscale("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    flat = (g.astype(np.int64) * Z + z)
    idx = torch.from_numpy(np.arange(NM)[:, None] * (G * Z) + flat[None, :]).cuda().reshape(-1)
    for var in (P.SJ_VAR_DIRECT, P.SJ_VAR_MFMA):
        print(f"case fp64 large variant={var}", flush=True)
        phi_d = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
        h = P.sj_specialize(P.SJ_LTIMES, layout="DGZ", Z=Z, G=G, D=D, NM=NM, variant=var)
        P.sj_run(h, [L_d, psi_d, phi_d])
        got = host(phi_d[idx]).reshape(NM, -1)
        assert componentwise_err(got, exact, scale) <= TOL_F64
        del phi_d
        torch.cuda.empty_cache()
    del psi_d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("cols_per_lane", [1, 4])
def test_bf16_accumulate_exact(P, orc, cols_per_lane):
    """SJ_FLAG_ACCUMULATE in BF16: small-integer inputs make every product and
    partial sum exact in FP32, so out0 + 2 L psi comes out bit for bit."""
    Z, G, D, NM = 64, 4, 32, 8
    rng = np.random.default_rng(5)
    Li = rng.integers(-4, 5, (NM, D)).astype(float)
    pi = rng.integers(0, 8, D * G * Z).astype(float)
    out0 = rng.integers(-50, 50, NM * G * Z).astype(np.float32)
    ref = orc.ltimes("DGZ", Z, G, D, NM, Li, pi)
    for dt in (P.SJ_BF16, P.SJ_BF16X3):
        phi_d = dev(out0.copy())
        h = P.sj_specialize(P.SJ_LTIMES, layout="DGZ", Z=Z, G=G, D=D, NM=NM, dtype=dt, tile_n=cols_per_lane,
                            flags=P.SJ_FLAG_ACCUMULATE)
        for _ in range(2):
            P.sj_run(h, [dev(Li), dev(pi.astype(np.float32)), phi_d])
        assert np.array_equal(host(phi_d).astype(np.float64), out0.astype(np.float64) + 2 * ref)
