"""Exhaustive autotuner for the moment contractions.

For a problem shape it enumerates a candidate set C(shape) of specializations
(kernel structure x tile parameters), compiles all of them in parallel on host
threads (each sj_specialize call releases the interpreter lock while hiprtc
runs), times each one with sj_time_run, and returns the fastest together with
every timing.  This is the profile-guided autotuning named as future work in
ClangJIT section 6; it is also the reference the learned picker is measured against.

The candidate set (at most 35 per kernel and layout):
  * innermost axis is a column axis (DGZ, DZG, GDZ, ZDG):
    DIRECT with tile_n (columns per thread) in {1, 2} dividing the contiguous
    extent, unroll in {4, 8, 16}, block in {256, 512}, order in {ascending,
    rotated}  (<= 24); FP64 MFMA column kernel with tile_n (columns per lane)
    in {1, 2, 4} dividing the extent and unroll (reduction steps per group of
    loads) in {2, 4, 8}, default order  (<= 9)
  * innermost axis is D (GZD, ZGD): STAGED with tile_k in {8, 16, 32},
    block 256, tile_n in {256, 512}; FP64 MFMA, ordinary or nontemporal
    loads (explicit flags), with operands read by every lane (order 1: 16-row tiles per wave
    in {1, 2, 4}, block in {256, 512}) or read as contiguous runs staged in
    LDS (order 2: tiles x block in {1x64, 1x256, 2x128, 2x256}, workgroups in
    the hardware's XCD order or renumbered so that each XCD takes a contiguous
    range of each sweep); DIRECT with tile_n 1, unroll 8  (<= 35)
  * BF16 dtypes: columns per lane in {1, 4} (4 when it divides the extent),
    block in {256, 512}  (<= 4)
Candidates that the specializer rejects for a shape (register or LDS limits)
are reported as rejected; candidates that resolve to the same specialization
as an earlier one are dropped.

Batched small products (bgemm_candidates, tune_bgemm): the workgroup form
(persistent, the waves of a workgroup share a window) with window elements
per array in {1024, 2048, 4096}, 16x16 tiles per work item in {1, 2, 4},
block in {512, 1024} and the next window prefetched or not; the wave form
(each wave owns a window) with windows of {256, 512} elements, {1, 2} tiles
per item, block 256  (<= 40).  Each candidate is timed on the caller's batch
through a plan, with the caller's scratch buffer read before every timed
launch so that the batch is read from HBM.
"""
from __future__ import annotations

import statistics
from concurrent.futures import ThreadPoolExecutor

from . import sj

LAYOUTS = sj.LAYOUTS


def bgemm_candidates() -> list:
    out = []
    for win in (1024, 2048, 4096):
        for u in (1, 2, 4):
            for block in (512, 1024):
                for order in (2, 1):
                    out.append(dict(variant=sj.SJ_VAR_MFMA, tile_n=win, unroll=u, block=block, order=order))
    for win in (256, 512):
        for u in (1, 2):
            out.append(dict(variant=sj.SJ_VAR_DIRECT, tile_n=win, unroll=u, block=256))
    return out


def tune_bgemm(n_host, A, B, C, cands=None, reps: int = 5, warmup: int = 1, flush=None, farm=None):
    """Time every batched-product candidate on the caller's batch (sizes
    n_host, device arrays A, B, C as for sj_batch_run).  ``flush`` (a device
    tensor) is read in full before every timed launch, so the batch comes from
    HBM.  Returns the same dict as tune_exhaustive."""
    import torch
    cands = bgemm_candidates() if cands is None else cands
    if farm is not None:
        made = farm.specialize_many([(sj.SJ_BGEMM, dict(c)) for c in cands])
        built = [(c, h, err) for c, (h, _, err) in zip(cands, made)]
    else:
        built = compile_all(sj.SJ_BGEMM, {}, cands, threads=1)
    stream = torch.cuda.current_stream()
    results, rejected = [], []
    for c, h, err in built:
        if h is None:
            rejected.append((c, str(err)))
            continue
        plan = sj.sj_batch_plan(h, n_host)
        try:
            for _ in range(warmup):
                sj.sj_batch_run(plan, A, B, C)
            ts = []
            for _ in range(reps):
                if flush is not None:
                    flush.sum()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                sj.sj_batch_run(plan, A, B, C)
                e1.record(stream)
                ts.append((e0, e1))
            torch.cuda.synchronize()
            t = [x.elapsed_time(y) for x, y in ts]
        finally:
            sj.sj_plan_destroy(plan)
        results.append((c, statistics.median(t), min(t)))
    if not results:
        raise RuntimeError(f"no batched-product candidate compiled: {rejected[:2]}")
    order = sorted(range(len(results)), key=lambda i: (results[i][1], i))
    best = results[order[0]]
    return dict(best=best[0], best_ms=best[1], results=results, rejected=rejected)


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
        return distinct(kernel, dict(layout=layout, Z=Z, G=G, D=D, NM=NM, dtype=dtype), out)
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
        for fl in (sj.SJ_FLAG_LOADS_CACHED, sj.SJ_FLAG_LOADS_NONTEMPORAL):
            for rt in (1, 2, 4):      # operands read by every lane straight from HBM
                for block in (256, 512):
                    out.append(dict(variant=sj.SJ_VAR_MFMA, tile_n=rt, block=block, order=1, flags=fl))
            for rt, block in ((1, 64), (1, 256), (2, 128), (2, 256)):   # contiguous runs staged in LDS
                for xcd in (sj.SJ_FLAG_XCD_INTERLEAVED, sj.SJ_FLAG_XCD_CONTIGUOUS):
                    out.append(dict(variant=sj.SJ_VAR_MFMA, tile_n=rt, block=block, order=2, flags=fl | xcd))
        out.append(dict(variant=sj.SJ_VAR_DIRECT, tile_n=1, unroll=8, block=256))
    return distinct(kernel, dict(layout=layout, Z=Z, G=G, D=D, NM=NM, dtype=dtype), out)


def distinct(kernel: int, base: dict, cands: list) -> list:
    """Drop candidates that resolve to the same specialization as an earlier
    one (a tile the specializer clamps, a policy that equals the default):
    the emitted source is the identity.  Candidates the specializer refuses are
    kept, to be reported as rejected."""
    seen, out = set(), []
    for c in cands:
        try:
            src = sj.sj_emit_source(kernel, **dict(base, **c))
        except sj.SJError:
            out.append(c)
            continue
        if src not in seen:
            seen.add(src)
            out.append(c)
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
