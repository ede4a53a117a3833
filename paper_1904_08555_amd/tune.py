"""Exhaustive autotuner for the moment contractions.

For a problem shape it enumerates a candidate set C(shape) of specializations
(kernel structure x tile parameters), compiles all of them in parallel on host
threads (each sj_specialize call releases the interpreter lock while hiprtc
runs), times each one with sj_time_run, and returns the fastest together with
every timing.  This is the profile-guided autotuning named as future work in
ClangJIT section 6; it is also the reference the learned picker is measured against.

The candidate set (at most 33 per kernel and layout):
  * innermost axis is a column axis (DGZ, DZG, GDZ, ZDG):
    DIRECT with tile_n (columns per thread) in {1, 2} dividing the contiguous
    extent, unroll in {4, 8, 16}, block in {256, 512}, order in {ascending,
    rotated}  (<= 24); FP64 MFMA column kernel with tile_n (columns per lane)
    in {1, 2, 4} dividing the extent and unroll (reduction steps per group of
    loads) in {2, 4, 8}, default order  (<= 9)
  * innermost axis is D (GZD, ZGD): STAGED with tile_k in {8, 16, 32},
    block 256, tile_n in {256, 512}; FP64 MFMA, ordinary or nontemporal
    loads, with operands read by every lane (order 1: 16-row tiles per wave
    in {1, 2, 4}, block in {256, 512}) or read as contiguous runs staged in
    LDS (order 2: tiles x block in {1x64, 1x256, 2x128, 2x256}); DIRECT with
    tile_n 1, unroll 8  (<= 27)
  * BF16 dtypes: columns per lane in {1, 4} (4 when it divides the extent),
    block in {256, 512}  (<= 4)
Candidates that the specializer rejects for a shape (register or LDS limits)
are dropped.
"""
from __future__ import annotations

import statistics
from concurrent.futures import ThreadPoolExecutor

from . import sj

LAYOUTS = sj.LAYOUTS


def contiguous_extent(layout: str, Z: int, G: int) -> int:
    return {"DGZ": G * Z, "DZG": G * Z, "GDZ": Z, "ZDG": G}.get(layout, 1)


def candidates(kernel: int, layout: str, Z: int, G: int, D: int, NM: int, dtype: int = sj.SJ_F64) -> list:
    out = []
    ext = contiguous_extent(layout, Z, G)
    if dtype != sj.SJ_F64:
        for cpl in (1, 4):
            if ext % cpl:
                continue
            for block in (256, 512):
                out.append(dict(variant=sj.SJ_VAR_MFMA, tile_n=cpl, block=block))
        return out
    if ext > 1:
        for vec in (1, 2):
            if ext % vec:
                continue
            for unroll in (4, 8, 16):
                for block in (256, 512):
                    for order in (1, 2):
                        out.append(dict(variant=sj.SJ_VAR_DIRECT, tile_n=vec, unroll=unroll, block=block,
                                        order=order))
        for cpl in (1, 2, 4):
            if ext % cpl:
                continue
            for pf in (2, 4, 8):
                out.append(dict(variant=sj.SJ_VAR_MFMA, tile_n=cpl, unroll=pf))
    else:
        for tk in (8, 16, 32):
            for tn in (256, 512):
                out.append(dict(variant=sj.SJ_VAR_STAGED, tile_n=tn, tile_k=tk, block=256))
        for fl in (0, sj.SJ_FLAG_LOADS_NONTEMPORAL):
            for rt in (1, 2, 4):      # operands read by every lane straight from HBM
                for block in (256, 512):
                    out.append(dict(variant=sj.SJ_VAR_MFMA, tile_n=rt, block=block, order=1, flags=fl))
            for rt, block in ((1, 64), (1, 256), (2, 128), (2, 256)):   # contiguous runs staged in LDS
                out.append(dict(variant=sj.SJ_VAR_MFMA, tile_n=rt, block=block, order=2, flags=fl))
        out.append(dict(variant=sj.SJ_VAR_DIRECT, tile_n=1, unroll=8, block=256))
    return out


def compile_all(kernel: int, base: dict, cands: list, threads: int = 8, compile_only: bool = False):
    """Specialize every candidate in parallel; returns [(cand, handle or None, error)]."""
    def one(c):
        spec = dict(base)
        spec.update(c)
        if compile_only:
            spec["flags"] = spec.get("flags", 0) | sj.SJ_FLAG_COMPILE_ONLY
        try:
            return c, sj.sj_specialize(kernel, **spec), None
        except sj.SJError as e:
            return c, None, e

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(one, cands))


def tune_exhaustive(kernel: int, layout: str, Z: int, G: int, D: int, NM: int, ptrs, dtype: int = sj.SJ_F64,
                    cands=None, reps: int = 10, warmup: int = 2, flush=None, threads: int = 8, farm=None):
    """Time every candidate on the caller's buffers ``ptrs`` (as for sj_run).
    Compiles on host threads, or in the worker processes of ``farm`` (a
    CompileFarm) when given.
    Returns dict(best=cand, best_ms=median, results=[(cand, median_ms, min_ms)], rejected=[...])."""
    base = dict(layout=layout, Z=Z, G=G, D=D, NM=NM, dtype=dtype)
    if cands is None:
        cands = candidates(kernel, layout, Z, G, D, NM, dtype)
    if farm is not None:
        made = farm.specialize_many([(kernel, dict(base, **c)) for c in cands])
        built = [(c, h, err) for c, (h, _, err) in zip(cands, made)]
    else:
        built = compile_all(kernel, base, cands, threads)
    results, rejected = [], []
    for c, h, err in built:
        if h is None:
            rejected.append((c, str(err)))
            continue
        t = sj.sj_time_run(h, ptrs, warmup=warmup, reps=reps, flush=flush)
        results.append((c, statistics.median(t), min(t)))
    if not results:
        raise RuntimeError(f"no candidate compiled for {base}: {rejected[:2]}")
    # lowest median, ties to the lowest candidate index
    order = sorted(range(len(results)), key=lambda i: (results[i][1], i))
    best = results[order[0]]
    return dict(best=best[0], best_ms=best[1], results=results, rejected=rejected)
