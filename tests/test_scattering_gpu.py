"""GPU parity of the scattering source kernel against the FP64 CPU oracle,
through the C ABI, over the six nestings.  Bar: componentwise
|gpu - oracle| <= 1e-12 * sum_g' |S||phi| (helpers.TOL_F64); bit-exact for
integer inputs.  Materials are laid out both in contiguous regions (the
wave-uniform matrix paths) and at random per zone (per-lane matrices)."""
import math

import numpy as np
import pytest

import sj_inputs as gen
from helpers import LAYOUTS, TOL_F64, componentwise_err, dev, host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1904_08555_amd as P
    P.sj_init(0)
    return P


def scat_inputs(seed, Z, G, NM, nmat, regions):
    rng = np.random.default_rng(seed)
    nl = math.isqrt(NM - 1) + 1
    S = rng.uniform(-1.0, 1.0, (nmat, nl, G, G))
    if regions:
        mat = ((np.arange(Z) * nmat) // Z).astype(np.int32)
    else:
        mat = rng.integers(0, nmat, Z).astype(np.int32)
    phi = rng.uniform(-1.0, 1.0, (NM, G, Z))
    return S, mat, phi


def run(P, layout, Z, G, NM, nmat, S, mat, phi_flat, order=0, **kw):
    out = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
    h = P.sj_specialize(P.SJ_SCATTERING, layout=layout, Z=Z, G=G, NM=NM, count=nmat, order=order, **kw)
    P.sj_run(h, [dev(S.ravel()), dev(mat), dev(phi_flat), out])
    return host(out)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shape", [(37, 5, 10, 3), (300, 3, 16, 2), (1, 1, 1, 1), (256, 32, 16, 4), (9, 4, 40, 2),
                                   (20, 3, 70, 2), (130, 64, 4, 1)], ids=lambda s: "Z%dG%dNM%dmat%d" % s)
@pytest.mark.parametrize("regions", [True, False], ids=["regions", "random"])
@pytest.mark.parametrize("variant", ["auto", "direct"])
def test_scattering_parity(P, orc, layout, shape, regions, variant):
    """The default structure (matrix cores where g or z is innermost and G <= 32) and the
    vector-FMA structure, on every nesting."""
    Z, G, NM, nmat = shape
    S, mat, phi = scat_inputs(41, Z, G, NM, nmat, regions)
    phi_flat = gen.to_layout(phi, layout).ravel()
    var = P.SJ_VAR_AUTO if variant == "auto" else P.SJ_VAR_DIRECT
    got = run(P, layout, Z, G, NM, nmat, S, mat, phi_flat, variant=var)
    ref = orc.scattering(layout, Z, G, NM, S, mat, phi_flat)
    scale = orc.scattering(layout, Z, G, NM, S, mat, phi_flat, absolute=True)
    assert componentwise_err(got, ref, scale) <= TOL_F64


@pytest.mark.parametrize("shape", [(37, 5, 10, 3), (300, 3, 16, 2), (1, 1, 1, 1), (256, 32, 16, 4), (9, 4, 40, 2)],
                         ids=lambda s: "Z%dG%dNM%dmat%d" % s)
@pytest.mark.parametrize("regions", [True, False], ids=["regions", "random"])
def test_scattering_parity_zdg_threads_along_nm(P, orc, shape, regions):
    """ZDG, vector-FMA structure with order 2: threads along nm, the material's degree
    matrices staged in LDS."""
    Z, G, NM, nmat = shape
    S, mat, phi = scat_inputs(47, Z, G, NM, nmat, regions)
    phi_flat = gen.to_layout(phi, "ZDG").ravel()
    d = P.SJ_VAR_DIRECT
    got = run(P, "ZDG", Z, G, NM, nmat, S, mat, phi_flat, order=2, variant=d)
    ref = orc.scattering("ZDG", Z, G, NM, S, mat, phi_flat)
    scale = orc.scattering("ZDG", Z, G, NM, S, mat, phi_flat, absolute=True)
    assert componentwise_err(got, ref, scale) <= TOL_F64
    # same sums in the same order as threads along z
    assert np.array_equal(got, run(P, "ZDG", Z, G, NM, nmat, S, mat, phi_flat, order=1, variant=d))


@pytest.mark.parametrize("layout", ["DGZ", "GZD", "ZDG"])
def test_scattering_integer_bitexact(P, orc, layout):
    Z, G, NM, nmat = 70, 12, 9, 3
    rng = np.random.default_rng(42)
    S = rng.integers(-4, 5, (nmat, 3, G, G)).astype(np.float64)
    mat = rng.integers(0, nmat, Z).astype(np.int32)
    phi_flat = gen.to_layout(rng.integers(0, 8, (NM, G, Z)).astype(np.float64), layout).ravel()
    got = run(P, layout, Z, G, NM, nmat, S, mat, phi_flat, variant=P.SJ_VAR_DIRECT)
    assert np.array_equal(got, orc.scattering(layout, Z, G, NM, S, mat, phi_flat))


def test_scattering_bad_material_gives_nan(P, orc):
    """Zones whose material index is out of range get NaN; the others are exact."""
    Z, G, NM, nmat = 50, 6, 4, 2
    S, mat, phi = scat_inputs(43, Z, G, NM, nmat, True)
    bad = np.array([3, 17, 49])
    mat_bad = mat.copy()
    mat_bad[bad] = [-1, 2, 1000]
    phi_flat = gen.to_layout(phi, "DGZ").ravel()
    got = gen.from_layout(run(P, "DGZ", Z, G, NM, nmat, S, mat_bad, phi_flat, variant=P.SJ_VAR_DIRECT), "DGZ", NM, G, Z)
    ref = gen.from_layout(orc.scattering("DGZ", Z, G, NM, S, mat, phi_flat), "DGZ", NM, G, Z)
    assert np.all(np.isnan(got[:, :, bad]))
    good = np.setdiff1d(np.arange(Z), bad)
    assert np.all(np.abs(got[:, :, good] - ref[:, :, good]) <= 1e-12 * 32)


def test_scattering_checks(P):
    Z, G, NM, nmat = 8, 2, 4, 1
    h = P.sj_specialize(P.SJ_SCATTERING, layout="DGZ", Z=Z, G=G, NM=NM, count=nmat)
    x = torch.zeros(4096, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SJError) as e:
        P.sj_run(h, [x, x, x])
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    with pytest.raises(P.SJError) as e:   # phi_out overlaps phi
        P.sj_run(h, [x, x.data_ptr() + 1024, x.data_ptr() + 2048, x.data_ptr() + 2048])
    assert e.value.status == P.SJ_ERR_ALIAS


@pytest.mark.parametrize("layout,order", [("DGZ", 0), ("ZGD", 0), ("ZDG", 0), ("ZDG", 2), ("DZG", 0)])
def test_scattering_full_size_sampled(P, orc, layout, order):
    """Z=32768 G=32 NM=16, four materials in contiguous zone regions, the vector-FMA
    structure: 512 sampled zones (all their lines) against the oracle on those zones."""
    Z, G, NM, nmat = 32768, 32, 16, 4
    S = np.random.default_rng(44).uniform(-1.0, 1.0, (nmat, 4, G, G))
    mat = ((np.arange(Z) * nmat) // Z).astype(np.int32)
    li = LAYOUTS.index(layout)
    phi_d = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
    from sj_inputs import device as gdev
    gdev.fill(phi_d, 0, gen.ARR_PHI, gdev.DIST_U01, li, (NM, G, Z))
    out = torch.empty_like(phi_d)
    h = P.sj_specialize(P.SJ_SCATTERING, layout=layout, Z=Z, G=G, NM=NM, count=nmat, order=order,
                        variant=P.SJ_VAR_DIRECT)
    P.sj_run(h, [dev(S.ravel()), dev(mat), phi_d, out])
    zs = np.sort(np.random.default_rng(45).choice(Z, 512, replace=False))
    zs[-1] = Z - 1
    phi_log = gen.from_layout(host(phi_d), layout, NM, G, Z)[:, :, zs]
    got_log = gen.from_layout(host(out), layout, NM, G, Z)[:, :, zs]
    sub = np.ascontiguousarray(phi_log)
    ref = orc.scattering("DGZ", len(zs), G, NM, S, mat[zs], sub.ravel()).reshape(NM, G, len(zs))
    scale = orc.scattering("DGZ", len(zs), G, NM, S, mat[zs], sub.ravel(), absolute=True).reshape(NM, G, len(zs))
    assert componentwise_err(got_log, ref, scale) <= TOL_F64
    del phi_d, out
    torch.cuda.empty_cache()


# ---- the FP64 matrix-core structure (g innermost: DZG, ZDG; z innermost: DGZ, GDZ) ----------

MFMA_LAYOUTS = ["DZG", "ZDG", "DGZ", "GDZ"]


@pytest.mark.parametrize("layout", MFMA_LAYOUTS)
@pytest.mark.parametrize("shape", [(37, 5, 10, 3), (300, 3, 16, 2), (1, 1, 1, 1), (256, 32, 16, 4), (9, 4, 40, 2),
                                   (20, 31, 7, 2), (130, 17, 4, 1), (48, 16, 5, 3), (1000, 32, 9, 4)],
                         ids=lambda s: "Z%dG%dNM%dmat%d" % s)
@pytest.mark.parametrize("regions", [True, False], ids=["regions", "random"])
@pytest.mark.parametrize("rt", [1, 2, 4])
@pytest.mark.parametrize("order", [1, 2])
def test_scattering_mfma_parity(P, orc, layout, shape, regions, rt, order):
    """16-zone tiles with ragged ends (Z not a multiple of 16), G not a multiple of 16,
    materials shared by a tile or mixed within it (one pass per material); tiles taken
    moments-outer (order 1) and zone-blocks-outer (order 2)."""
    Z, G, NM, nmat = shape
    S, mat, phi = scat_inputs(53, Z, G, NM, nmat, regions)
    phi_flat = gen.to_layout(phi, layout).ravel()
    got = run(P, layout, Z, G, NM, nmat, S, mat, phi_flat, variant=P.SJ_VAR_MFMA, tile_n=rt, order=order)
    ref = orc.scattering(layout, Z, G, NM, S, mat, phi_flat)
    scale = orc.scattering(layout, Z, G, NM, S, mat, phi_flat, absolute=True)
    assert componentwise_err(got, ref, scale) <= TOL_F64


@pytest.mark.parametrize("layout", MFMA_LAYOUTS + ["GZD", "ZGD"])
def test_scattering_mfma_integer_bitexact_and_bad_material(P, orc, layout):
    """Small integers: every partial sum is exact, so the matrix-core result equals the
    oracle's bit for bit; zones with an out-of-range material get NaN, the rest stay exact."""
    Z, G, NM, nmat = 70, 12, 9, 3
    rng = np.random.default_rng(42)
    S = rng.integers(-4, 5, (nmat, 3, G, G)).astype(np.float64)
    mat = rng.integers(0, nmat, Z).astype(np.int32)
    phi_flat = gen.to_layout(rng.integers(0, 8, (NM, G, Z)).astype(np.float64), layout).ravel()
    ref = orc.scattering(layout, Z, G, NM, S, mat, phi_flat)
    got = run(P, layout, Z, G, NM, nmat, S, mat, phi_flat, variant=P.SJ_VAR_MFMA)
    assert np.array_equal(got, ref)
    bad = np.array([0, 17, 33, 69])
    mat_bad = mat.copy()
    mat_bad[bad] = [-1, nmat, 1000, -7]
    got = gen.from_layout(run(P, layout, Z, G, NM, nmat, S, mat_bad, phi_flat, variant=P.SJ_VAR_MFMA), layout, NM, G, Z)
    ref_l = gen.from_layout(ref, layout, NM, G, Z)
    assert np.all(np.isnan(got[:, :, bad]))
    good = np.setdiff1d(np.arange(Z), bad)
    assert np.array_equal(got[:, :, good], ref_l[:, :, good])


@pytest.mark.parametrize("layout", MFMA_LAYOUTS + ["GZD", "ZGD"])
@pytest.mark.parametrize("regions", [True, False], ids=["regions", "random"])
def test_scattering_mfma_full_size_sampled(P, orc, layout, regions):
    """Z=32768 G=32 NM=16, four materials: 512 sampled zones (all their lines) against the oracle."""
    Z, G, NM, nmat = 32768, 32, 16, 4
    S = np.random.default_rng(44).uniform(-1.0, 1.0, (nmat, 4, G, G))
    mat = (((np.arange(Z) * nmat) // Z) if regions else np.random.default_rng(46).integers(0, nmat, Z)).astype(np.int32)
    li = LAYOUTS.index(layout)
    phi_d = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
    from sj_inputs import device as gdev
    gdev.fill(phi_d, 0, gen.ARR_PHI, gdev.DIST_U01, li, (NM, G, Z))
    out = torch.empty_like(phi_d)
    h = P.sj_specialize(P.SJ_SCATTERING, layout=layout, Z=Z, G=G, NM=NM, count=nmat, variant=P.SJ_VAR_MFMA)
    P.sj_run(h, [dev(S.ravel()), dev(mat), phi_d, out])
    zs = np.sort(np.random.default_rng(45).choice(Z, 512, replace=False))
    zs[-1] = Z - 1
    phi_log = gen.from_layout(host(phi_d), layout, NM, G, Z)[:, :, zs]
    got_log = gen.from_layout(host(out), layout, NM, G, Z)[:, :, zs]
    sub = np.ascontiguousarray(phi_log)
    ref = orc.scattering("DGZ", len(zs), G, NM, S, mat[zs], sub.ravel()).reshape(NM, G, len(zs))
    scale = orc.scattering("DGZ", len(zs), G, NM, S, mat[zs], sub.ravel(), absolute=True).reshape(NM, G, len(zs))
    assert componentwise_err(got_log, ref, scale) <= TOL_F64
    del phi_d, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("layout", ["GZD", "ZGD"])
@pytest.mark.parametrize("shape", [(37, 5, 10, 3), (300, 3, 16, 2), (256, 32, 16, 4), (9, 4, 40, 2),
                                   (20, 31, 7, 2), (130, 17, 4, 1), (48, 16, 5, 3), (1000, 32, 9, 4), (17, 2, 2, 2)],
                         ids=lambda s: "Z%dG%dNM%dmat%d" % s)
@pytest.mark.parametrize("regions", [True, False], ids=["regions", "random"])
@pytest.mark.parametrize("block", [256, 512])
def test_scattering_mfma_blocks_parity(P, orc, layout, shape, regions, block):
    """nm innermost: 16-zone blocks staged whole in LDS, one tile per moment; ragged zone blocks,
    odd NM (8-byte pieces), G not a multiple of 16, materials mixed inside a block."""
    Z, G, NM, nmat = shape
    S, mat, phi = scat_inputs(59, Z, G, NM, nmat, regions)
    phi_flat = gen.to_layout(phi, layout).ravel()
    got = run(P, layout, Z, G, NM, nmat, S, mat, phi_flat, variant=P.SJ_VAR_MFMA, block=block)
    ref = orc.scattering(layout, Z, G, NM, S, mat, phi_flat)
    scale = orc.scattering(layout, Z, G, NM, S, mat, phi_flat, absolute=True)
    assert componentwise_err(got, ref, scale) <= TOL_F64
