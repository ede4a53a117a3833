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


def run(P, layout, Z, G, NM, nmat, S, mat, phi_flat, order=0):
    out = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
    h = P.sj_specialize(P.SJ_SCATTERING, layout=layout, Z=Z, G=G, NM=NM, count=nmat, order=order)
    P.sj_run(h, [dev(S.ravel()), dev(mat), dev(phi_flat), out])
    return host(out)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shape", [(37, 5, 10, 3), (300, 3, 16, 2), (1, 1, 1, 1), (256, 32, 16, 4), (9, 4, 40, 2),
                                   (20, 3, 70, 2), (130, 64, 4, 1)], ids=lambda s: "Z%dG%dNM%dmat%d" % s)
@pytest.mark.parametrize("regions", [True, False], ids=["regions", "random"])
def test_scattering_parity(P, orc, layout, shape, regions):
    Z, G, NM, nmat = shape
    S, mat, phi = scat_inputs(41, Z, G, NM, nmat, regions)
    phi_flat = gen.to_layout(phi, layout).ravel()
    got = run(P, layout, Z, G, NM, nmat, S, mat, phi_flat)
    ref = orc.scattering(layout, Z, G, NM, S, mat, phi_flat)
    scale = orc.scattering(layout, Z, G, NM, S, mat, phi_flat, absolute=True)
    assert componentwise_err(got, ref, scale) <= TOL_F64


@pytest.mark.parametrize("shape", [(37, 5, 10, 3), (300, 3, 16, 2), (1, 1, 1, 1), (256, 32, 16, 4), (9, 4, 40, 2)],
                         ids=lambda s: "Z%dG%dNM%dmat%d" % s)
@pytest.mark.parametrize("regions", [True, False], ids=["regions", "random"])
def test_scattering_parity_zdg_threads_along_nm(P, orc, shape, regions):
    """ZDG with order 2: threads along nm, the material's degree matrices staged in LDS."""
    Z, G, NM, nmat = shape
    S, mat, phi = scat_inputs(47, Z, G, NM, nmat, regions)
    phi_flat = gen.to_layout(phi, "ZDG").ravel()
    got = run(P, "ZDG", Z, G, NM, nmat, S, mat, phi_flat, order=2)
    ref = orc.scattering("ZDG", Z, G, NM, S, mat, phi_flat)
    scale = orc.scattering("ZDG", Z, G, NM, S, mat, phi_flat, absolute=True)
    assert componentwise_err(got, ref, scale) <= TOL_F64
    assert np.array_equal(got, run(P, "ZDG", Z, G, NM, nmat, S, mat, phi_flat, order=1))   # same sums, same order


@pytest.mark.parametrize("layout", ["DGZ", "GZD", "ZDG"])
def test_scattering_integer_bitexact(P, orc, layout):
    Z, G, NM, nmat = 70, 12, 9, 3
    rng = np.random.default_rng(42)
    S = rng.integers(-4, 5, (nmat, 3, G, G)).astype(np.float64)
    mat = rng.integers(0, nmat, Z).astype(np.int32)
    phi_flat = gen.to_layout(rng.integers(0, 8, (NM, G, Z)).astype(np.float64), layout).ravel()
    got = run(P, layout, Z, G, NM, nmat, S, mat, phi_flat)
    assert np.array_equal(got, orc.scattering(layout, Z, G, NM, S, mat, phi_flat))


def test_scattering_bad_material_gives_nan(P, orc):
    """Zones whose material index is out of range get NaN; the others are exact."""
    Z, G, NM, nmat = 50, 6, 4, 2
    S, mat, phi = scat_inputs(43, Z, G, NM, nmat, True)
    bad = np.array([3, 17, 49])
    mat_bad = mat.copy()
    mat_bad[bad] = [-1, 2, 1000]
    phi_flat = gen.to_layout(phi, "DGZ").ravel()
    got = gen.from_layout(run(P, "DGZ", Z, G, NM, nmat, S, mat_bad, phi_flat), "DGZ", NM, G, Z)
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
    """Z=32768 G=32 NM=16, four materials in contiguous zone regions: 512
    sampled zones (all their lines) against the oracle on those zones."""
    Z, G, NM, nmat = 32768, 32, 16, 4
    S = np.random.default_rng(44).uniform(-1.0, 1.0, (nmat, 4, G, G))
    mat = ((np.arange(Z) * nmat) // Z).astype(np.int32)
    li = LAYOUTS.index(layout)
    phi_d = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
    from sj_inputs import device as gdev
    gdev.fill(phi_d, 0, gen.ARR_PHI, gdev.DIST_U01, li, (NM, G, Z))
    out = torch.empty_like(phi_d)
    h = P.sj_specialize(P.SJ_SCATTERING, layout=layout, Z=Z, G=G, NM=NM, count=nmat, order=order)
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
