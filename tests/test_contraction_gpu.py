"""GPU parity of LTimes / LPlusTimes (specialized and generic kernels) against
the FP64 CPU oracle, through the C ABI.  Bar: componentwise
|gpu - oracle| <= 1e-12 * sum|L||psi| (helpers.TOL_F64); bit-exact where the
inputs make every partial sum exact."""
import numpy as np
import pytest

import sj_inputs as gen
from sj_inputs import device as gdev
from sj_inputs import quadrature as quad

from helpers import LAYOUTS, TOL_F64, componentwise_err, contraction_inputs, dev, host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1904_08555_amd as P
    P.sj_init(0)
    return P


def run_ltimes(P, layout, Z, G, D, NM, L_d, psi_d, generic=False, **tile):
    """generic: False (specialized), True (generic kernel), "layout" (generic kernel compiled per nesting)."""
    phi_d = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
    if generic:
        fl = P.SJ_FLAG_GENERIC_PER_LAYOUT if generic == "layout" else 0
        P.sj_generic_run(P.SJ_LTIMES, [L_d, psi_d, phi_d], layout=layout, Z=Z, G=G, D=D, NM=NM, flags=fl)
    else:
        h = P.sj_specialize(P.SJ_LTIMES, layout=layout, Z=Z, G=G, D=D, NM=NM, **tile)
        P.sj_run(h, [L_d, psi_d, phi_d])
    return phi_d


def run_lplus(P, layout, Z, G, D, NM, Lp_d, phi_d, generic=False, **tile):
    out_d = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
    if generic:
        fl = P.SJ_FLAG_GENERIC_PER_LAYOUT if generic == "layout" else 0
        P.sj_generic_run(P.SJ_LPLUSTIMES, [Lp_d, phi_d, out_d], layout=layout, Z=Z, G=G, D=D, NM=NM, flags=fl)
    else:
        h = P.sj_specialize(P.SJ_LPLUSTIMES, layout=layout, Z=Z, G=G, D=D, NM=NM, **tile)
        P.sj_run(h, [Lp_d, phi_d, out_d])
    return out_d


SMALL = [
    (37, 5, 11, 6),     # ragged everywhere
    (300, 3, 48, 16),   # several tiles + tail
    (1, 1, 1, 1),
    (1, 7, 5, 3),       # Z = 1
    (129, 1, 9, 4),     # G = 1
    (64, 2, 1, 5),      # D = 1
    (50, 4, 7, 1),      # NM = 1
]


@pytest.mark.parametrize("generic", [False, True, "layout"], ids=["jit", "generic", "generic_per_layout"])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shape", SMALL, ids=lambda s: "Z%dG%dD%dNM%d" % s)
def test_ltimes_lplustimes_small(P, orc, layout, shape, generic):
    Z, G, D, NM = shape
    print(f"case layout={layout} shape={shape} generic={generic}", flush=True)
    L, Lp, psi, phi_in = contraction_inputs(3, layout, Z, G, D, NM)
    ref = orc.ltimes(layout, Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)
    got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), generic))
    assert componentwise_err(got, ref, scale) <= TOL_F64
    ref2 = orc.lplustimes(layout, Z, G, D, NM, Lp, phi_in)
    # sum_nm |L+[d,nm]| |phi[nm]|: the oracle's abs-scale with the roles of D and NM swapped
    scale2 = orc.ltimes_absscale(layout, Z, G, NM, D, Lp, phi_in)
    got2 = host(run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi_in), generic))
    assert componentwise_err(got2, ref2, scale2) <= TOL_F64


@pytest.mark.parametrize("layout", ["DGZ", "ZDG", "GZD"])
@pytest.mark.parametrize("tile", [dict(tile_n=1, unroll=3, block=64), dict(tile_n=4, unroll=16, block=512),
                                  dict(tile_n=2, unroll=1, block=1024), dict(tile_n=2, unroll=3, order=2),
                                  dict(tile_n=1, unroll=2, block=64, order=2)],
                         ids=["t1u3b64", "t4u16b512", "t2u1b1024", "t2u3rot", "t1u2b64rot"])
def test_direct_tiles(P, orc, layout, tile):
    Z, G, D, NM = 96, 4, 13, 6
    L, Lp, psi, phi_in = contraction_inputs(5, layout, Z, G, D, NM)
    if layout == "GZD" and tile["tile_n"] != 1:
        pytest.skip("D-innermost layouts have a contiguous column extent of 1")
    ref = orc.ltimes(layout, Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)
    got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), variant=P.SJ_VAR_DIRECT, **tile))
    assert componentwise_err(got, ref, scale) <= TOL_F64
    ref2 = orc.lplustimes(layout, Z, G, D, NM, Lp, phi_in)
    scale2 = orc.ltimes_absscale(layout, Z, G, NM, D, Lp, phi_in)
    got2 = host(run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi_in), variant=P.SJ_VAR_DIRECT, **tile))
    assert componentwise_err(got2, ref2, scale2) <= TOL_F64


@pytest.mark.parametrize("layout", ["GZD", "ZGD"])
@pytest.mark.parametrize("tile", [dict(tile_n=64, tile_k=5, block=64), dict(tile_n=512, tile_k=16, block=256),
                                  dict(tile_n=256, tile_k=40, block=128)], ids=["n64k5", "n512k16", "n256k40"])
def test_staged_tiles(P, orc, layout, tile):
    Z, G, D, NM = 150, 3, 37, 9
    L, Lp, psi, phi_in = contraction_inputs(6, layout, Z, G, D, NM)
    ref = orc.ltimes(layout, Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)
    got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), variant=P.SJ_VAR_STAGED, **tile))
    assert componentwise_err(got, ref, scale) <= TOL_F64
    ref2 = orc.lplustimes(layout, Z, G, D, NM, Lp, phi_in)
    scale2 = orc.ltimes_absscale(layout, Z, G, NM, D, Lp, phi_in)
    got2 = host(run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi_in), variant=P.SJ_VAR_STAGED, **tile))
    assert componentwise_err(got2, ref2, scale2) <= TOL_F64


@pytest.mark.parametrize("layout", LAYOUTS)
def test_onehot_and_integer_bitexact(P, orc, layout):
    """One-hot L gives a bit-exact row gather; integer inputs are exact in any order."""
    Z, G, D, NM = 70, 3, 10, 4
    psi = gen.to_layout(gen.psi_logical(1, D, G, Z), layout).ravel()
    L = np.zeros((NM, D))
    L[np.arange(NM), [9, 0, 4, 4]] = 1.0
    got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi)))
    assert np.array_equal(got, orc.ltimes(layout, Z, G, D, NM, L, psi))
    rng = np.random.default_rng(2)
    Li = rng.integers(-4, 5, (NM, D)).astype(float)
    pi = rng.integers(0, 8, D * G * Z).astype(float)
    got = host(run_ltimes(P, layout, Z, G, D, NM, dev(Li), dev(pi)))
    assert np.array_equal(got, orc.ltimes(layout, Z, G, D, NM, Li, pi))
    Lpi = rng.integers(-4, 5, (D, NM)).astype(float)
    phii = rng.integers(-7, 8, NM * G * Z).astype(float)
    got = host(run_lplus(P, layout, Z, G, D, NM, dev(Lpi), dev(phii)))
    assert np.array_equal(got, orc.lplustimes(layout, Z, G, D, NM, Lpi, phii))


@pytest.mark.parametrize("DNM", [(48, 16), (96, 16)])
def test_quadrature_roundtrip(P, DNM):
    """L * L+ = I on a matching quadrature: LTimes(LPlusTimes(phi)) = phi on the GPU."""
    D, NM = DNM
    lmax, a, b = quad.SETS[DNM]
    L, Lp = quad.moment_matrices(lmax, a, b)
    Z, G = 333, 4
    for layout in ("DGZ", "ZDG", "ZGD"):
        phi = gen.sym(4, gen.ARR_PHI, np.arange(NM * G * Z, dtype=np.uint64))
        psi_d = run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi))
        back = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), psi_d))
        assert np.abs(back - phi).max() < 1e-13


def test_fill_matches_host_generator(P):
    """The device fill kernel reproduces the host generator bit for bit."""
    D, G, Z = 6, 5, 7
    for layout in range(6):
        t = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
        gdev.fill(t, 123, gen.ARR_PSI, gdev.DIST_U01, layout, (D, G, Z))
        ref = gen.to_layout(gen.psi_logical(123, D, G, Z), LAYOUTS[layout]).ravel()
        assert np.array_equal(host(t), ref)
    t = torch.empty(1000, dtype=torch.float64, device="cuda")
    gdev.fill(t, 7, gen.ARR_L, gdev.DIST_SYM)
    assert np.array_equal(host(t), gen.sym(7, gen.ARR_L, np.arange(1000, dtype=np.uint64)))
    t = torch.empty(1000, dtype=torch.float32, device="cuda")
    gdev.fill(t, 7, gen.ARR_PSI, gdev.DIST_U01_24)
    assert np.array_equal(host(t).astype(np.float64), gen.u01_24(7, gen.ARR_PSI, np.arange(1000, dtype=np.uint64)))


def test_config_dgz_small_full(P, orc):
    """LTimes + LPlusTimes, DGZ, Z=4096 G=8 D=48 NM=16: every output checked."""
    Z, G, D, NM = 4096, 8, 48, 16
    L, Lp, psi, _ = contraction_inputs(0, "DGZ", Z, G, D, NM)
    phi_ref = orc.ltimes("DGZ", Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale("DGZ", Z, G, D, NM, L, psi)
    phi_d = run_ltimes(P, "DGZ", Z, G, D, NM, dev(L), dev(psi))
    assert componentwise_err(host(phi_d), phi_ref, scale) <= TOL_F64
    # LPlusTimes consumes the oracle's phi, so errors do not compound
    out_ref = orc.lplustimes("DGZ", Z, G, D, NM, Lp, phi_ref)
    scale2 = orc.ltimes_absscale("DGZ", Z, G, NM, D, Lp, phi_ref)
    got = host(run_lplus(P, "DGZ", Z, G, D, NM, dev(Lp), dev(phi_ref)))
    assert componentwise_err(got, out_ref, scale2) <= TOL_F64


@pytest.mark.parametrize("layout", LAYOUTS)
def test_six_layouts_full_size_sampled(P, orc, layout):
    """Z=32768 G=32 D=96 NM=16 in every nesting, launched as the benchmark
    launches it; 4096 sampled columns checked against the oracle one by one."""
    Z, G, D, NM = 32768, 32, 96, 16
    li = LAYOUTS.index(layout)
    psi_d = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
    gdev.fill(psi_d, 0, gen.ARR_PSI, gdev.DIST_U01, li, (D, G, Z))
    L = gen.matrix_sym(0, gen.ARR_L, NM, D)
    Lp = gen.matrix_sym(0, gen.ARR_LPLUS, D, NM)
    phi_d = run_ltimes(P, layout, Z, G, D, NM, dev(L), psi_d)
    out_d = run_lplus(P, layout, Z, G, D, NM, dev(Lp), phi_d)
    rng = np.random.default_rng(li)
    g = rng.integers(0, G, 4096)
    z = rng.integers(0, Z, 4096)
    g[:2], z[:2] = [0, G - 1], [0, Z - 1]
    cols = gen.psi_columns(0, D, G, Z, g, z)                        # (D, S)
    ref = orc.ltimes("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    scale = orc.ltimes_absscale("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    phi_log = gen.from_layout(host(phi_d), layout, NM, G, Z)
    assert componentwise_err(phi_log[:, g, z], ref, scale) <= TOL_F64
    # LPlusTimes on the GPU's own phi: compare with the oracle applied to those same phi columns
    phi_cols = phi_log[:, g, z]
    ref2 = orc.lplustimes("DGZ", len(g), 1, D, NM, Lp, phi_cols).reshape(D, -1)
    scale2 = orc.ltimes_absscale("DGZ", len(g), 1, NM, D, Lp, phi_cols).reshape(D, -1)
    out_log = gen.from_layout(host(out_d), layout, D, G, Z)
    assert componentwise_err(out_log[:, g, z], ref2, scale2) <= TOL_F64
    del psi_d, phi_d, out_d
    torch.cuda.empty_cache()


def test_generic_full_size_sampled(P, orc):
    Z, G, D, NM = 32768, 32, 96, 16
    for layout, mode in (("DGZ", True), ("GZD", True), ("DGZ", "layout"), ("ZGD", "layout")):
        li = LAYOUTS.index(layout)
        psi_d = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
        gdev.fill(psi_d, 0, gen.ARR_PSI, gdev.DIST_U01, li, (D, G, Z))
        L = gen.matrix_sym(0, gen.ARR_L, NM, D)
        phi_d = run_ltimes(P, layout, Z, G, D, NM, dev(L), psi_d, generic=mode)
        rng = np.random.default_rng(9)
        g = rng.integers(0, G, 1024)
        z = rng.integers(0, Z, 1024)
        cols = gen.psi_columns(0, D, G, Z, g, z)
        ref = orc.ltimes("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
        scale = orc.ltimes_absscale("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
        phi_log = gen.from_layout(host(phi_d), layout, NM, G, Z)
        assert componentwise_err(phi_log[:, g, z], ref, scale) <= TOL_F64
        del psi_d, phi_d
    torch.cuda.empty_cache()


def test_run_checks(P):
    """Null, misaligned and aliased pointers are rejected before launch."""
    Z, G, D, NM = 64, 2, 8, 4
    h = P.sj_specialize(P.SJ_LTIMES, layout="DGZ", Z=Z, G=G, D=D, NM=NM)
    L = torch.zeros(NM * D, dtype=torch.float64, device="cuda")
    psi = torch.zeros(D * G * Z + 2, dtype=torch.float64, device="cuda")
    phi = torch.zeros(NM * G * Z, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SJError) as e:
        P.sj_run(h, [L, psi.data_ptr() + 8, phi])
    assert e.value.status == P.SJ_ERR_ALIGN
    with pytest.raises(P.SJError) as e:
        P.sj_run(h, [L, psi, psi.data_ptr() + 16 * 8])
    assert e.value.status == P.SJ_ERR_ALIAS
    with pytest.raises(P.SJError) as e:
        P.sj_run(h, [L, 0, phi])
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    with pytest.raises(P.SJError) as e:
        P.sj_run(h, [L, psi])
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    P.sj_run(h, [L, psi, phi])
    torch.cuda.synchronize()


def test_same_key_same_handle_and_stats(P):
    s0 = P.sj_stats()
    h1 = P.sj_specialize(P.SJ_LTIMES, layout="ZDG", Z=33, G=16, D=12, NM=5)
    h2 = P.sj_specialize(P.SJ_LTIMES, layout="zdg", Z=33, G=16, D=12, NM=5, block=256, unroll=8, tile_n=2)
    assert h1 == h2
    s1 = P.sj_stats()
    assert s1["compiles"] - s0["compiles"] <= 1 and s1["hits"] - s0["hits"] >= 1
    info = P.sj_handle_info(h1)
    assert info["kernel_name"] == "sj_ltimes_direct_zdg" and info["load_ms"] > 0 and info["scratch_bytes"] == 0


MFMA_SHAPES = [(150, 3, 37, 9), (64, 4, 96, 16), (33, 1, 5, 3), (16, 1, 16, 16), (40, 2, 17, 20), (7, 3, 128, 64),
               (150, 3, 38, 10), (21, 5, 24, 18)]


@pytest.mark.parametrize("layout", ["GZD", "ZGD"])
@pytest.mark.parametrize("shape", MFMA_SHAPES, ids=lambda s: "Z%dG%dD%dNM%d" % s)
@pytest.mark.parametrize("tile", [dict(), dict(tile_n=1, block=64), dict(tile_n=2, block=512), dict(tile_n=4, block=128),
                                  dict(order=1), dict(tile_n=2, block=64, order=2), dict(tile_n=1, block=512, order=2)],
                         ids=["default", "t1b64", "t2b512", "t4b128", "o1", "t2b64o2", "t1b512o2"])
def test_mfma64_rows(P, orc, layout, shape, tile):
    """FP64 matrix-core row kernels (D innermost), both operand paths (order 1:
    lanes read rows directly; order 2: contiguous runs staged through LDS,
    even D and NM only): ragged rows, odd and non-multiple-of-16 reduction
    lengths, output counts not multiple of 16, weights in registers and in LDS
    (D=128, NM=64)."""
    Z, G, D, NM = shape
    L, Lp, psi, phi_in = contraction_inputs(8, layout, Z, G, D, NM)
    try:
        got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), variant=P.SJ_VAR_MFMA, **tile))
    except P.SJError as e:
        assert e.status == P.SJ_ERR_UNSUPPORTED, e
        got = None
    if got is not None:
        ref = orc.ltimes(layout, Z, G, D, NM, L, psi)
        scale = orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)
        assert componentwise_err(got, ref, scale) <= TOL_F64
    try:
        got2 = host(run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi_in), variant=P.SJ_VAR_MFMA, **tile))
    except P.SJError as e:
        assert e.status == P.SJ_ERR_UNSUPPORTED, e
        return
    ref2 = orc.lplustimes(layout, Z, G, D, NM, Lp, phi_in)
    scale2 = orc.ltimes_absscale(layout, Z, G, NM, D, Lp, phi_in)
    assert componentwise_err(got2, ref2, scale2) <= TOL_F64


@pytest.mark.parametrize("layout", ["GZD", "ZGD"])
@pytest.mark.parametrize("shape", [(150, 3, 38, 10), (64, 4, 96, 16), (21, 5, 24, 18), (1, 1, 2, 2)],
                         ids=lambda s: "Z%dG%dD%dNM%d" % s)
@pytest.mark.parametrize("tile", [dict(tile_n=1), dict(tile_n=2, block=64)], ids=["t1", "t2b64"])
def test_mfma64_rows_orders_bitwise(P, layout, shape, tile):
    """The LDS-staged row kernel (order 2) runs the MFMA sequences of the
    direct row kernel (order 1): identical results, bit for bit, for LTimes,
    LPlusTimes and accumulation."""
    Z, G, D, NM = shape
    L, Lp, psi, phi_in = contraction_inputs(20, layout, Z, G, D, NM)
    L_d, Lp_d, psi_d, phi_d = dev(L), dev(Lp), dev(psi), dev(phi_in)
    for kern, W_d, x_d, n_out in ((P.SJ_LTIMES, L_d, psi_d, NM), (P.SJ_LPLUSTIMES, Lp_d, phi_d, D)):
        outs = []
        for order in (1, 2):
            for flags in (0, P.SJ_FLAG_ACCUMULATE):
                h = P.sj_specialize(kern, layout=layout, Z=Z, G=G, D=D, NM=NM, variant=P.SJ_VAR_MFMA, order=order,
                                    flags=flags, **tile)
                assert P.sj_handle_info(h)["kernel_name"].endswith(("_lds_" if order == 2 else "_mfma_") + layout.lower())
                o = torch.full((n_out * G * Z,), 0.25, dtype=torch.float64, device="cuda")
                P.sj_run(h, [W_d, x_d, o])
                outs.append(host(o))
        assert np.array_equal(outs[0], outs[2]) and np.array_equal(outs[1], outs[3])


def test_mfma64_full_size_sampled(P, orc):
    Z, G, D, NM = 32768, 32, 96, 16
    layout = "ZGD"
    li = LAYOUTS.index(layout)
    psi_d = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
    gdev.fill(psi_d, 0, gen.ARR_PSI, gdev.DIST_U01, li, (D, G, Z))
    L = gen.matrix_sym(0, gen.ARR_L, NM, D)
    Lp = gen.matrix_sym(0, gen.ARR_LPLUS, D, NM)
    phi_d = run_ltimes(P, layout, Z, G, D, NM, dev(L), psi_d, variant=P.SJ_VAR_MFMA)
    out_d = run_lplus(P, layout, Z, G, D, NM, dev(Lp), phi_d, variant=P.SJ_VAR_MFMA)
    rng = np.random.default_rng(11)
    g = rng.integers(0, G, 2048)
    z = rng.integers(0, Z, 2048)
    g[-1], z[-1] = G - 1, Z - 1
    cols = gen.psi_columns(0, D, G, Z, g, z)
    ref = orc.ltimes("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    scale = orc.ltimes_absscale("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    phi_log = gen.from_layout(host(phi_d), layout, NM, G, Z)
    assert componentwise_err(phi_log[:, g, z], ref, scale) <= TOL_F64
    phi_cols = phi_log[:, g, z]
    ref2 = orc.lplustimes("DGZ", len(g), 1, D, NM, Lp, phi_cols).reshape(D, -1)
    scale2 = orc.ltimes_absscale("DGZ", len(g), 1, NM, D, Lp, phi_cols).reshape(D, -1)
    out_log = gen.from_layout(host(out_d), layout, D, G, Z)
    assert componentwise_err(out_log[:, g, z], ref2, scale2) <= TOL_F64
    del psi_d, phi_d, out_d
    torch.cuda.empty_cache()


COLS_SHAPES = [(37, 5, 11, 6), (300, 3, 48, 16), (64, 4, 96, 16), (40, 2, 17, 20), (7, 3, 128, 64), (16, 8, 5, 3),
               (1, 1, 1, 1)]


@pytest.mark.parametrize("layout", ["DGZ", "DZG", "GDZ", "ZDG"])
@pytest.mark.parametrize("shape", COLS_SHAPES, ids=lambda s: "Z%dG%dD%dNM%d" % s)
@pytest.mark.parametrize("tile", [dict(), dict(tile_n=1, unroll=1, block=64), dict(tile_n=2, unroll=3, order=2),
                                  dict(tile_n=4, unroll=16, block=512, order=2), dict(tile_n=4, unroll=2, order=1)],
                         ids=["default", "t1p1b64", "t2p3rot", "t4p16b512rot", "t4p2"])
def test_mfma64_cols(P, orc, layout, shape, tile):
    """FP64 matrix-core column kernels (a column axis innermost): ragged column
    tiles, reduction lengths not multiple of 4, ragged last group, output
    counts not multiple of 16, rotated group order, W in 64 KiB of LDS."""
    Z, G, D, NM = shape
    print(f"case cols layout={layout} shape={shape} tile={tile}", flush=True)
    L, Lp, psi, phi_in = contraction_inputs(9, layout, Z, G, D, NM)
    _, I = {"DGZ": (1, G * Z), "DZG": (1, G * Z), "GDZ": (G, Z), "ZDG": (Z, G)}[layout]
    if I == 1:
        # a contiguous extent of 1 is a row contraction: the specializer takes the
        # FP64 MFMA row kernel (its tiles are covered by test_mfma64_rows)
        h = P.sj_specialize(P.SJ_LTIMES, layout=layout, Z=Z, G=G, D=D, NM=NM, variant=P.SJ_VAR_MFMA)
        assert "rows_mfma" in P.sj_handle_info(h)["kernel_name"]
        tile = {}
    t = tile.get("tile_n", 0)
    if t and I % t:
        with pytest.raises(P.SJError) as e:
            run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), variant=P.SJ_VAR_MFMA, **tile)
        assert e.value.status == P.SJ_ERR_INVALID_ARG
        return
    got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), variant=P.SJ_VAR_MFMA, **tile))
    ref = orc.ltimes(layout, Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)
    assert componentwise_err(got, ref, scale) <= TOL_F64
    got2 = host(run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi_in), variant=P.SJ_VAR_MFMA, **tile))
    ref2 = orc.lplustimes(layout, Z, G, D, NM, Lp, phi_in)
    scale2 = orc.ltimes_absscale(layout, Z, G, NM, D, Lp, phi_in)
    assert componentwise_err(got2, ref2, scale2) <= TOL_F64


def test_mfma64_cols_onehot_bitexact(P, orc):
    """One-hot L through the column kernel: phi is a row gather of psi, bit for bit."""
    Z, G, D, NM = 300, 3, 48, 16
    layout = "DGZ"
    _, _, psi, _ = contraction_inputs(4, layout, Z, G, D, NM)
    L = np.zeros((NM, D))
    perm = np.random.default_rng(2).permutation(D)[:NM]
    L[np.arange(NM), perm] = 1.0
    got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L.ravel()), dev(psi), variant=P.SJ_VAR_MFMA))
    assert np.array_equal(got, orc.ltimes(layout, Z, G, D, NM, L.ravel(), psi))


@pytest.mark.parametrize("layout", ["DGZ", "ZDG"])
def test_mfma64_cols_full_size_sampled(P, orc, layout):
    """Z=32768 G=32 D=96 NM=16 through the column kernel (rotated order for
    DGZ, whose rows are 8 MiB apart), 2048 sampled columns checked."""
    Z, G, D, NM = 32768, 32, 96, 16
    li = LAYOUTS.index(layout)
    psi_d = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
    gdev.fill(psi_d, 0, gen.ARR_PSI, gdev.DIST_U01, li, (D, G, Z))
    L = gen.matrix_sym(0, gen.ARR_L, NM, D)
    Lp = gen.matrix_sym(0, gen.ARR_LPLUS, D, NM)
    phi_d = run_ltimes(P, layout, Z, G, D, NM, dev(L), psi_d, variant=P.SJ_VAR_MFMA)
    out_d = run_lplus(P, layout, Z, G, D, NM, dev(Lp), phi_d, variant=P.SJ_VAR_MFMA)
    rng = np.random.default_rng(12)
    g = rng.integers(0, G, 2048)
    z = rng.integers(0, Z, 2048)
    g[-1], z[-1] = G - 1, Z - 1
    cols = gen.psi_columns(0, D, G, Z, g, z)
    ref = orc.ltimes("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    scale = orc.ltimes_absscale("DGZ", len(g), 1, D, NM, L, cols).reshape(NM, -1)
    phi_log = gen.from_layout(host(phi_d), layout, NM, G, Z)
    assert componentwise_err(phi_log[:, g, z], ref, scale) <= TOL_F64
    phi_cols = phi_log[:, g, z]
    ref2 = orc.lplustimes("DGZ", len(g), 1, D, NM, Lp, phi_cols).reshape(D, -1)
    scale2 = orc.ltimes_absscale("DGZ", len(g), 1, NM, D, Lp, phi_cols).reshape(D, -1)
    out_log = gen.from_layout(host(out_d), layout, D, G, Z)
    assert componentwise_err(out_log[:, g, z], ref2, scale2) <= TOL_F64
    del psi_d, phi_d, out_d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("layout,variant", [("DGZ", 1), ("DGZ", 3), ("GDZ", 1), ("ZGD", 3), ("ZGD", 2)],
                         ids=["direct-dgz", "cols-dgz", "direct-gdz", "rows-zgd", "staged-zgd"])
def test_policy_flags_bitwise_identical(P, orc, layout, variant):
    """The load/store policy changes only the memory instructions: every
    combination gives the default's output bit for bit (and the default
    meets the oracle bar)."""
    Z, G, D, NM = 300, 3, 48, 16
    L, Lp, psi, phi_in = contraction_inputs(12, layout, Z, G, D, NM)
    ref = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), variant=variant))
    assert componentwise_err(ref, orc.ltimes(layout, Z, G, D, NM, L, psi),
                             orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)) <= TOL_F64
    ref2 = host(run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi_in), variant=variant))
    for lf in (P.SJ_FLAG_LOADS_CACHED, P.SJ_FLAG_LOADS_NONTEMPORAL):
        for sf in (P.SJ_FLAG_STORES_CACHED, P.SJ_FLAG_STORES_NONTEMPORAL):
            got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), variant=variant, flags=lf | sf))
            assert np.array_equal(got, ref), (lf, sf)
            got2 = host(run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi_in), variant=variant, flags=lf | sf))
            assert np.array_equal(got2, ref2), (lf, sf)


@pytest.mark.parametrize("layout,spec", [
    ("DGZ", dict(variant=1)), ("ZDG", dict(variant=1, tile_n=1)), ("DGZ", dict(variant=3)), ("GDZ", dict(variant=3)),
    ("ZGD", dict(variant=3)), ("GZD", dict(variant=2)), ("DZG", dict(variant=1, order=2, tile_n=2, unroll=4))],
    ids=["direct-dgz", "direct-zdg", "cols-dgz", "cols-gdz", "rows-zgd", "staged-gzd", "direct-dzg-rot"])
def test_index64_forced_small(P, orc, layout, spec):
    """64-bit indexing (chosen automatically for arrays of 2^31 elements and
    more) forced at a small shape for every structure: the same results."""
    Z, G, D, NM = 300, 3, 48, 16
    L, Lp, psi, phi_in = contraction_inputs(13, layout, Z, G, D, NM)
    spec = dict(spec, flags=P.SJ_FLAG_INDEX64)
    got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), **spec))
    assert componentwise_err(got, orc.ltimes(layout, Z, G, D, NM, L, psi),
                             orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)) <= TOL_F64
    got2 = host(run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi_in), **spec))
    assert componentwise_err(got2, orc.lplustimes(layout, Z, G, D, NM, Lp, phi_in),
                             orc.ltimes_absscale(layout, Z, G, NM, D, Lp, phi_in)) <= TOL_F64
    h = P.sj_specialize(P.SJ_LTIMES, layout=layout, Z=Z, G=G, D=D, NM=NM, **spec)
    assert "typedef long long sj_index_t" in P.sj_emit_source(P.SJ_LTIMES, layout=layout, Z=Z, G=G, D=D, NM=NM,
                                                               **spec)
    assert P.sj_handle_info(h)["scratch_bytes"] == 0


@pytest.mark.parametrize("shape", [(64, 2, 4096, 2), (33, 3, 4096, 5), (40, 2, 8, 128), (7, 5, 3, 128)],
                         ids=["D4096NM2", "D4096NM5", "D8NM128", "D3NM128"])
@pytest.mark.parametrize("layout", ["DGZ", "ZDG", "GZD"])
def test_edge_sizes(P, orc, layout, shape):
    """The largest reduction length (D = 4096) and the largest moment count a
    column keeps in registers (NM = 128), through the default structures and
    the generic kernels; a structure that declines a shape says so."""
    Z, G, D, NM = shape
    L, Lp, psi, phi_in = contraction_inputs(14, layout, Z, G, D, NM)
    ref = orc.ltimes(layout, Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)
    ref2 = orc.lplustimes(layout, Z, G, D, NM, Lp, phi_in)
    scale2 = orc.ltimes_absscale(layout, Z, G, NM, D, Lp, phi_in)
    for generic in (False, True):
        print(f"case edge layout={layout} shape={shape} generic={generic}", flush=True)
        try:
            got = host(run_ltimes(P, layout, Z, G, D, NM, dev(L), dev(psi), generic))
            assert componentwise_err(got, ref, scale) <= TOL_F64
        except P.SJError as e:
            assert not generic and e.status == P.SJ_ERR_UNSUPPORTED, e
        try:
            got2 = host(run_lplus(P, layout, Z, G, D, NM, dev(Lp), dev(phi_in), generic))
            assert componentwise_err(got2, ref2, scale2) <= TOL_F64
        except P.SJError as e:
            assert not generic and e.status == P.SJ_ERR_UNSUPPORTED, e


@pytest.mark.parametrize("layout,spec", [
    ("DGZ", dict(variant=1)), ("DGZ", dict(variant=3)), ("GDZ", dict(variant=1)), ("ZDG", dict(variant=3)),
    ("ZGD", dict(variant=3)), ("GZD", dict(variant=2)), ("DZG", dict(variant=1, order=2, tile_n=2, unroll=4))],
    ids=["direct-dgz", "cols-dgz", "direct-gdz", "cols-zdg", "rows-zgd", "staged-gzd", "direct-dzg"])
def test_accumulate(P, orc, layout, spec):
    """SJ_FLAG_ACCUMULATE: out += result on every structure.  Bar: the FP64
    componentwise bound widened by the one extra addition,
    |got - (out0 + oracle)| <= 1e-12 (sum|L||psi| + |out0|)."""
    Z, G, D, NM = 300, 3, 48, 16
    L, Lp, psi, phi_in = contraction_inputs(15, layout, Z, G, D, NM)
    init = gen.sym(15, gen.ARR_PHI + 10, np.arange(max(NM, D) * G * Z, dtype=np.uint64))
    spec = dict(spec)
    spec["flags"] = spec.get("flags", 0) | P.SJ_FLAG_ACCUMULATE
    out0 = init[:NM * G * Z].copy()
    phi_d = dev(out0)
    h = P.sj_specialize(P.SJ_LTIMES, layout=layout, Z=Z, G=G, D=D, NM=NM, **spec)
    P.sj_run(h, [dev(L), dev(psi), phi_d])
    P.sj_run(h, [dev(L), dev(psi), phi_d])       # two direction sets summed
    ref = orc.ltimes(layout, Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)
    assert componentwise_err(host(phi_d), out0 + 2 * ref, 2 * scale + np.abs(out0)) <= TOL_F64
    out1 = init[:D * G * Z].copy()
    o_d = dev(out1)
    h2 = P.sj_specialize(P.SJ_LPLUSTIMES, layout=layout, Z=Z, G=G, D=D, NM=NM, **spec)
    P.sj_run(h2, [dev(Lp), dev(phi_in), o_d])
    ref2 = orc.lplustimes(layout, Z, G, D, NM, Lp, phi_in)
    scale2 = orc.ltimes_absscale(layout, Z, G, NM, D, Lp, phi_in)
    assert componentwise_err(host(o_d), out1 + ref2, scale2 + np.abs(out1)) <= TOL_F64


def test_accumulate_refused_where_unsupported(P):
    with pytest.raises(P.SJError) as e:
        P.sj_specialize(P.SJ_BGEMM, flags=P.SJ_FLAG_ACCUMULATE)
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SJError) as e:
        P.sj_generic_run(P.SJ_LTIMES, [x, x, x], layout="DGZ", Z=2, G=2, D=2, NM=2, flags=P.SJ_FLAG_ACCUMULATE)
    assert e.value.status == P.SJ_ERR_UNSUPPORTED


def run_fused(P, layout, Z, G, D, NM, L_d, Lp_d, psi_d, want_phi=True, **tile):
    out_d = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
    phi_d = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda") if want_phi else None
    h = P.sj_specialize(P.SJ_LTIMES_LPLUS, layout=layout, Z=Z, G=G, D=D, NM=NM, **tile)
    P.sj_run(h, [L_d, Lp_d, psi_d, out_d] + ([phi_d] if want_phi else []))
    return out_d, phi_d


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shape", [(37, 5, 11, 6), (300, 3, 48, 16), (1, 1, 1, 1), (64, 2, 96, 16), (9, 4, 7, 40)],
                         ids=lambda s: "Z%dG%dD%dNM%d" % s)
def test_fused_ltimes_lplus(P, orc, layout, shape):
    """psi' = L+ (L psi) in one pass, against the oracle's two steps.  Bar:
    |psi'_gpu - psi'_oracle| <= 1e-12 * sum_nm |L+[d,nm]| sum_d' |L[nm,d']| |psi[d']|
    (phi's own error carried through L+), and phi to the LTimes bar."""
    Z, G, D, NM = shape
    L, Lp, psi, _ = contraction_inputs(16, layout, Z, G, D, NM)
    ref_phi = orc.ltimes(layout, Z, G, D, NM, L, psi)
    s_phi = orc.ltimes_absscale(layout, Z, G, D, NM, L, psi)
    ref_out = orc.lplustimes(layout, Z, G, D, NM, Lp, ref_phi)
    s_out = orc.ltimes_absscale(layout, Z, G, NM, D, Lp, s_phi)
    out_d, phi_d = run_fused(P, layout, Z, G, D, NM, dev(L), dev(Lp), dev(psi))
    assert componentwise_err(host(phi_d), ref_phi, s_phi) <= TOL_F64
    assert componentwise_err(host(out_d), ref_out, s_out) <= TOL_F64
    out2, _ = run_fused(P, layout, Z, G, D, NM, dev(L), dev(Lp), dev(psi), want_phi=False)
    assert np.array_equal(host(out2), host(out_d))       # the phi store does not change psi'


@pytest.mark.parametrize("layout,tile", [("DGZ", dict(tile_n=2, unroll=4, order=2)), ("ZDG", dict(tile_n=1, unroll=8)),
                                         ("GDZ", dict(tile_n=2, unroll=16, block=512))])
def test_fused_matches_separate_bitwise(P, layout, tile):
    """The fused kernel takes the separate DIRECT kernels' steps: with the same
    tiles, phi equals LTimes' output and psi' equals LPlusTimes applied to that
    phi, bit for bit."""
    Z, G, D, NM = 300, 4, 48, 16
    L, Lp, psi, _ = contraction_inputs(17, layout, Z, G, D, NM)
    L_d, Lp_d, psi_d = dev(L), dev(Lp), dev(psi)
    out_d, phi_d = run_fused(P, layout, Z, G, D, NM, L_d, Lp_d, psi_d, variant=1, **tile)
    phi_sep = run_ltimes(P, layout, Z, G, D, NM, L_d, psi_d, variant=1, **tile)
    out_sep = run_lplus(P, layout, Z, G, D, NM, Lp_d, phi_sep, variant=1, **tile)
    assert np.array_equal(host(phi_d), host(phi_sep))
    assert np.array_equal(host(out_d), host(out_sep))


@pytest.mark.parametrize("layout,tile", [("ZGD", dict(tile_n=2)), ("GZD", dict(tile_n=1)), ("ZGD", dict(tile_n=4, block=512)),
                                         ("GZD", dict(tile_n=2, block=64)), ("ZGD", dict(tile_n=1, order=1)),
                                         ("GZD", dict(tile_n=2, block=128, order=2))])
@pytest.mark.parametrize("shape", [(300, 4, 48, 16), (37, 3, 11, 21), (37, 3, 10, 22), (5, 3, 2, 2)],
                         ids=lambda s: "Z%dG%dD%dNM%d" % s)
def test_fused_rows_matches_separate_bitwise(P, layout, tile, shape):
    """D innermost: the fused matrix-core row kernel runs the separate row
    kernels' MFMA sequences (phase 2 reads the moments from LDS instead of HBM),
    so with the same tiles phi and psi' equal theirs bit for bit, ragged D and
    NM included."""
    Z, G, D, NM = shape
    if tile.get("order") == 2 and (D % 2 or NM % 2):
        pytest.skip("order 2 needs even D and NM")
    L, Lp, psi, _ = contraction_inputs(19, layout, Z, G, D, NM)
    L_d, Lp_d, psi_d = dev(L), dev(Lp), dev(psi)
    out_d, phi_d = run_fused(P, layout, Z, G, D, NM, L_d, Lp_d, psi_d, variant=3, **tile)
    phi_sep = run_ltimes(P, layout, Z, G, D, NM, L_d, psi_d, variant=3, **tile)
    out_sep = run_lplus(P, layout, Z, G, D, NM, Lp_d, phi_sep, variant=3, **tile)
    assert np.array_equal(host(phi_d), host(phi_sep))
    assert np.array_equal(host(out_d), host(out_sep))


def test_fused_checks(P):
    Z, G, D, NM = 8, 2, 4, 3
    x = torch.zeros(4096, dtype=torch.float64, device="cuda")
    h = P.sj_specialize(P.SJ_LTIMES_LPLUS, layout="DGZ", Z=Z, G=G, D=D, NM=NM)
    with pytest.raises(P.SJError) as e:   # psi_out overlaps psi
        P.sj_run(h, [x, x.data_ptr() + 1024, x.data_ptr() + 2048, x.data_ptr() + 2048])
    assert e.value.status == P.SJ_ERR_ALIAS
    with pytest.raises(P.SJError) as e:
        P.sj_run(h, [x, x, x])
    assert e.value.status == P.SJ_ERR_INVALID_ARG


@pytest.mark.parametrize("layout", ["DGZ", "ZGD"])
def test_fused_full_size_sampled(P, orc, layout):
    """Z=32768 G=32 D=96 NM=16, fused, 2048 sampled columns against the oracle's
    two steps on those columns."""
    Z, G, D, NM = 32768, 32, 96, 16
    li = LAYOUTS.index(layout)
    psi_d = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
    gdev.fill(psi_d, 0, gen.ARR_PSI, gdev.DIST_U01, li, (D, G, Z))
    L = gen.matrix_sym(0, gen.ARR_L, NM, D)
    Lp = gen.matrix_sym(0, gen.ARR_LPLUS, D, NM)
    out_d, phi_d = run_fused(P, layout, Z, G, D, NM, dev(L), dev(Lp), psi_d)
    rng = np.random.default_rng(18)
    g = rng.integers(0, G, 2048)
    z = rng.integers(0, Z, 2048)
    g[-1], z[-1] = G - 1, Z - 1
    cols = gen.psi_columns(0, D, G, Z, g, z)
    ref_phi = orc.ltimes("DGZ", len(g), 1, D, NM, L, cols)
    s_phi = orc.ltimes_absscale("DGZ", len(g), 1, D, NM, L, cols)
    ref_out = orc.lplustimes("DGZ", len(g), 1, D, NM, Lp, ref_phi).reshape(D, -1)
    s_out = orc.ltimes_absscale("DGZ", len(g), 1, NM, D, Lp, s_phi).reshape(D, -1)
    out_log = gen.from_layout(host(out_d), layout, D, G, Z)
    assert componentwise_err(out_log[:, g, z], ref_out, s_out) <= TOL_F64
    phi_log = gen.from_layout(host(phi_d), layout, NM, G, Z)
    assert componentwise_err(phi_log[:, g, z], ref_phi.reshape(NM, -1), s_phi.reshape(NM, -1)) <= TOL_F64
    del psi_d, out_d, phi_d
    torch.cuda.empty_cache()
