"""The exhaustive tuner's candidate space and selection rule, on the host.

The candidate set must be well formed at the shapes the benchmark and the
picker use (every candidate passes the specializer's validation, no two name
the same specialization), and the selection must be the argmin of the median
timings with ties to the lowest candidate index.  Timing itself needs the GPU
(tests/test_tune_gpu.py)."""
import json

import pytest

import paper_1904_08555_amd as P
from paper_1904_08555_amd import tune

SHAPES = [(32768, 32, 96, 16), (4096, 8, 48, 16), (27000, 100, 256, 64), (512, 9, 16, 4), (1000, 13, 40, 9)]


def canonical(kid, layout, shape, c):
    """The specialization a candidate resolves to: its emitted source."""
    Z, G, D, NM = shape
    return P.sj_emit_source(kid, layout=layout, Z=Z, G=G, D=D, NM=NM, **c)


@pytest.mark.parametrize("shape", SHAPES)
def test_candidates_valid_and_distinct(shape):
    Z, G, D, NM = shape
    for kid in (P.SJ_LTIMES, P.SJ_LPLUSTIMES):
        for lay in P.LAYOUTS:
            cands = tune.candidates(kid, lay, Z, G, D, NM)
            assert cands, (kid, lay, shape)
            assert len({json.dumps(c, sort_keys=True) for c in cands}) == len(cands)
            srcs = []
            for c in cands:
                try:
                    srcs.append(canonical(kid, lay, shape, c))
                except P.SJError as e:
                    # only resource limits may refuse a candidate, never a malformed tile
                    assert e.status == P.SJ_ERR_UNSUPPORTED, (kid, lay, shape, c, e)
            assert srcs, (kid, lay, shape)
            assert len(set(srcs)) == len(srcs), f"two candidates emit the same kernel: {kid} {lay} {shape}"


def test_every_candidate_accepted_at_six_nesting_shape():
    """At Z=32768 G=32 D=96 NM=16 nothing is refused: the benchmark's tuning
    times the whole space."""
    Z, G, D, NM = 32768, 32, 96, 16
    for kid in (P.SJ_LTIMES, P.SJ_LPLUSTIMES):
        for lay in P.LAYOUTS:
            for c in tune.candidates(kid, lay, Z, G, D, NM):
                canonical(kid, lay, (Z, G, D, NM), c)


def test_selection_is_argmin_of_medians(monkeypatch):
    """Fake compiles and timings: the lowest median wins, ties go to the
    lowest candidate index, refused candidates are reported, not timed."""
    cands = [dict(tile_n=1), dict(tile_n=2), dict(tile_n=4), dict(tile_n=3)]
    times = {1: [3.0, 1.0, 2.0], 2: [1.5, 1.5, 9.0], 4: [0.1, 1.5, 1.5]}

    def fake_compile_all(kernel, base, cs, threads=8, compile_only=False):
        return [(c, None, "refused") if c["tile_n"] == 3 else (c, c["tile_n"], None) for c in cs]

    def fake_time(h, ptrs, warmup=2, reps=10, flush=None, stream=None):
        return list(times[h])

    monkeypatch.setattr(tune, "compile_all", fake_compile_all)
    monkeypatch.setattr(tune.sj, "sj_time_run", fake_time)
    r = tune.tune_exhaustive(P.SJ_LTIMES, "DGZ", 8, 8, 8, 4, [], cands=cands)
    # medians: 2.0, 1.5, 1.5 -> tie between index 1 and 2, the lower index wins
    assert r["best"] == dict(tile_n=2) and r["best_ms"] == 1.5
    assert [c for c, _, _ in r["results"]] == cands[:3]
    assert [m for _, m, _ in r["results"]] == [2.0, 1.5, 1.5]
    assert [mn for _, _, mn in r["results"]] == [1.0, 1.5, 0.1]
    assert r["rejected"] == [(dict(tile_n=3), "refused")]
