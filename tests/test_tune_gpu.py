"""Full-size parity of every specialization the exhaustive tuner can choose, and
the tuner's own contract.

The benchmark times, per nesting and kernel, the tuner's winner over
tune.candidates, or (after its in-step refinement) one of the three best, the
library default, or, for LTimes, one of those with ordinary instead of
nontemporal stores.  Every one of those specializations is run here at the
six-nesting shape Z=32768 G=32 D=96 NM=16 (D = 96 exercises the unroll-16
rotated DIRECT body, the two-tile LDS-staged row kernel and every other tile
form the tuner enumerates) and checked on 1024 sampled columns against the
oracle to the FP64 bar."""
import numpy as np
import pytest

import sj_inputs as gen
from sj_inputs import device as gdev

from helpers import LAYOUTS, TOL_F64, componentwise_err, gather_columns, sample_columns

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

Z, G, D, NM = 32768, 32, 96, 16
NS = 1024


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1904_08555_amd as P
    P.sj_init(0)
    return P


@pytest.fixture(scope="module")
def farm():
    from paper_1904_08555_amd.farm import CompileFarm
    f = CompileFarm(12)
    yield f
    f.close()


@pytest.fixture(scope="module")
def ref(orc):
    """Oracle values on the sampled columns (the logical values are the same in
    every nesting, so one reference serves all six)."""
    g, z = sample_columns(11, G, Z, NS)
    L = gen.matrix_sym(0, gen.ARR_L, NM, D)
    Lp = gen.matrix_sym(0, gen.ARR_LPLUS, D, NM)
    psi_cols = gen.psi_columns(0, D, G, Z, g, z)                                   # (D, NS)
    nm = np.arange(NM, dtype=np.uint64)[:, None]
    phi_cols = gen.sym(0, gen.ARR_PHI, (nm * np.uint64(G) + g[None, :].astype(np.uint64)) * np.uint64(Z)
                       + z[None, :].astype(np.uint64))                             # (NM, NS)
    return dict(
        g=g, z=z, L=L, Lp=Lp,
        phi=orc.ltimes("DGZ", NS, 1, D, NM, L, psi_cols).reshape(NM, NS),
        phi_scale=orc.ltimes_absscale("DGZ", NS, 1, D, NM, L, psi_cols).reshape(NM, NS),
        psi_out=orc.lplustimes("DGZ", NS, 1, D, NM, Lp, phi_cols).reshape(D, NS),
        psi_out_scale=orc.ltimes_absscale("DGZ", NS, 1, NM, D, Lp, phi_cols).reshape(D, NS))


@pytest.fixture(scope="module")
def bufs(P, ref):
    b = dict(L=torch.from_numpy(ref["L"]).cuda(), Lp=torch.from_numpy(ref["Lp"]).cuda(),
             psi=torch.empty(D * G * Z, dtype=torch.float64, device="cuda"),
             phi=torch.empty(NM * G * Z, dtype=torch.float64, device="cuda"),
             out=torch.empty(D * G * Z, dtype=torch.float64, device="cuda"))
    yield b
    b.clear()
    torch.cuda.empty_cache()


def timed_space(P, tune, kid, layout):
    """Every spec the benchmark can time for (kernel, nesting)."""
    cands = tune.candidates(kid, layout, Z, G, D, NM) + [{}]
    if kid == P.SJ_LTIMES:
        # the in-step refinement also tries ordinary stores of phi
        extra = []
        for c in cands:
            c2 = dict(c)
            c2["flags"] = (c2.get("flags", 0) & ~P.SJ_FLAG_STORES_NONTEMPORAL) | P.SJ_FLAG_STORES_CACHED
            extra.append(c2)
        cands = cands + extra
    return cands


@pytest.mark.parametrize("kname", ["ltimes", "lplustimes"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_every_tuner_candidate_full_size(P, farm, ref, bufs, layout, kname):
    from paper_1904_08555_amd import tune
    li = LAYOUTS.index(layout)
    if kname == "ltimes":
        kid = P.SJ_LTIMES
        gdev.fill(bufs["psi"], 0, gen.ARR_PSI, gdev.DIST_U01, li, (D, G, Z))
        src, dst, W, A = bufs["psi"], bufs["phi"], bufs["L"], NM
        want, scale = ref["phi"], ref["phi_scale"]
    else:
        kid = P.SJ_LPLUSTIMES
        gdev.fill(bufs["phi"], 0, gen.ARR_PHI, gdev.DIST_SYM, li, (NM, G, Z))
        src, dst, W, A = bufs["phi"], bufs["out"], bufs["Lp"], D
        want, scale = ref["psi_out"], ref["psi_out_scale"]
    cands = timed_space(P, tune, kid, layout)
    base = dict(layout=layout, Z=Z, G=G, D=D, NM=NM)
    made = farm.specialize_many([(kid, dict(base, **c)) for c in cands])
    worst = 0.0
    for c, (h, _, err) in zip(cands, made):
        # the tuner only enumerates specializations that run at this shape
        assert h is not None, f"{kname} {layout} {c}: {err}"
        dst.fill_(float("nan"))
        P.sj_run(h, [W, src, dst])
        got = gather_columns(dst, layout, A, G, Z, ref["g"], ref["z"])
        e = componentwise_err(got, want, scale)
        assert e <= TOL_F64, f"{kname} {layout} {c}: componentwise error {e}"
        worst = max(worst, e)
    print(f"{kname} {layout}: {len(cands)} specializations, worst componentwise error {worst:.2e}")


def test_tune_exhaustive_contract(P, orc):
    """tune_exhaustive times every candidate it can compile, reports the ones
    the specializer refuses, and returns the lowest median (ties to the lowest
    index) whose handle computes the oracle's result."""
    from paper_1904_08555_amd import tune
    from helpers import contraction_inputs, dev, host
    Zs, Gs, Ds, NMs = 4096, 8, 48, 16
    L, _, psi, _ = contraction_inputs(0, "DGZ", Zs, Gs, Ds, NMs)
    L_d, psi_d = dev(L), dev(psi)
    phi_d = torch.empty(NMs * Gs * Zs, dtype=torch.float64, device="cuda")
    cands = tune.candidates(P.SJ_LTIMES, "DGZ", Zs, Gs, Ds, NMs)
    bad = dict(variant=P.SJ_VAR_DIRECT, tile_n=3)          # columns per thread must be 1, 2 or 4
    r = tune.tune_exhaustive(P.SJ_LTIMES, "DGZ", Zs, Gs, Ds, NMs, [L_d, psi_d, phi_d], cands=cands + [bad],
                             reps=3, warmup=1, threads=4)
    assert len(r["results"]) == len(cands)
    assert [c for c, _ in r["rejected"]] == [bad]
    meds = [m for _, m, _ in r["results"]]
    i = min(range(len(meds)), key=lambda k: (meds[k], k))
    assert r["best"] == r["results"][i][0] and r["best_ms"] == meds[i]
    assert all(mn <= m for _, m, mn in r["results"])
    h = P.sj_specialize(P.SJ_LTIMES, layout="DGZ", Z=Zs, G=Gs, D=Ds, NM=NMs, **r["best"])
    phi_d.fill_(float("nan"))
    P.sj_run(h, [L_d, psi_d, phi_d])
    want = orc.ltimes("DGZ", Zs, Gs, Ds, NMs, L, psi)
    scale = orc.ltimes_absscale("DGZ", Zs, Gs, Ds, NMs, L, psi)
    assert componentwise_err(host(phi_d), want, scale) <= TOL_F64
