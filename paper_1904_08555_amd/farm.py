"""Parallel compilation across worker processes.

hiprtc serializes compiles inside one process (measured: 8 threads compiling
8 keys took as long as compiling them one after another), so the autotuner and
the picker's data collection spread compiles over spawned worker processes.
Each worker runs sj_specialize with SJ_FLAG_COMPILE_ONLY (no GPU work) and
returns the code object; the parent adopts it with sj_specialize_with_code,
which fills the same cache entry a local compile would.
"""
from __future__ import annotations

import multiprocessing as mp

from . import sj


def _worker_init():
    sj.lib()


def _compile_one(item):
    kernel, spec = item
    spec = dict(spec)
    spec["flags"] = int(spec.get("flags", 0)) | sj.SJ_FLAG_COMPILE_ONLY
    try:
        h = sj.sj_specialize(kernel, **spec)
        return sj.sj_handle_code(h), sj.sj_handle_info(h)["compile_ms"], None
    except sj.SJError as e:
        return None, 0.0, (e.status, e.message)


class CompileFarm:
    """Pool of `workers` compile processes (spawned, so they share no state
    with the parent's GPU context)."""

    def __init__(self, workers: int = 8):
        self.workers = max(1, int(workers))
        ctx = mp.get_context("spawn")
        self.pool = ctx.Pool(self.workers, initializer=_worker_init)

    def close(self):
        if self.pool is not None:
            self.pool.close()
            self.pool.join()
            self.pool = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def compile(self, items, log=None, every: int = 250):
        """items: [(kernel, spec dict)] -> [(code bytes or None, compile_ms, error or None)].
        With `log`, reports progress every `every` finished compiles."""
        items = list(items)
        out = []
        for i, r in enumerate(self.pool.imap(_compile_one, items, chunksize=1)):
            out.append(r)
            if log and (i + 1) % every == 0:
                log(f"compiled {i + 1}/{len(items)}")
        return out

    def specialize_many(self, items, log=None):
        """Compile `items` in the workers and adopt each result in this process.
        Returns [(handle or None, compile_ms, error)] in the order of `items`."""
        out = []
        for (kernel, spec), (code, ms, err) in zip(items, self.compile(items, log=log)):
            if code is None:
                out.append((None, ms, err))
                continue
            try:
                h = sj.sj_specialize_with_code(kernel, code, **spec)
                out.append((h, ms, None))
            except sj.SJError as e:
                out.append((None, ms, (e.status, e.message)))
        return out
