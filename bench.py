#!/usr/bin/env python3
"""Benchmark: runtime-specialized LTimes / LPlusTimes on one MI355X.

Workload (default): all six nestings DGZ, DZG, GDZ, GZD, ZDG, ZGD chosen at run
time, FP64, Z = 32^3 = 32768 zones, G = 32 groups, D = 96 directions,
NM = 16 moments; psi ~ U[0,1), L and L+ ~ U[-1,1), seed 0 (counter-based
generator, values identical across layouts).  One step = for every nesting: the
specialization lookup (cache hit), LTimes psi -> phi, and LPlusTimes phi -> psi'.
All inputs are resident in HBM before the timed region; each array is 805 MB
or 134 MB, larger than the 256 MB last-level cache, so every step streams HBM.

Printed: one JSON line (metric, value = algorithmic GB/s of the whole step,
roofline of the dominant kernel from live HIP-event timing, the CPU oracle
baseline on a bounded sample, and the generic-kernel comparison).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LTimes GB/s & %roofline: JIT-specialized vs generic kernel; JIT ms; picker regret"
HBM_PEAK_GBS = 8000.0
LAYOUTS = ("DGZ", "DZG", "GDZ", "GZD", "ZDG", "ZGD")


def algorithmic_bytes(Z, G, D, NM, esz=8):
    """Each operand read once, each result written once (LTimes or LPlusTimes)."""
    return (D + NM) * G * Z * esz + NM * D * 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--Z", type=int, default=32768)
    ap.add_argument("--G", type=int, default=32)
    ap.add_argument("--D", type=int, default=96)
    ap.add_argument("--NM", type=int, default=16)
    ap.add_argument("--layouts", default=",".join(LAYOUTS))
    ap.add_argument("--no-generic", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the CPU baseline sample")
    ap.add_argument("--tile", default="", help="override tile params, e.g. 'tile_n=2,unroll=8,block=256'")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {a.gpus}); "
              "the contractions are independent per (g, z) column, so N GPUs would each run the one-GPU kernel "
              "on a zone shard.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1904_08555_amd as P
    import sj_inputs as gen
    from sj_inputs import device as gdev

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.sj_init(0)
    Z, G, D, NM = a.Z, a.G, a.D, a.NM
    layouts = [x for x in a.layouts.split(",") if x]
    tile = {}
    for kv in filter(None, a.tile.split(",")):
        k, v = kv.split("=")
        tile[k] = int(v)
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream

    L_d = torch.empty(NM * D, dtype=torch.float64, device="cuda")
    Lp_d = torch.empty(D * NM, dtype=torch.float64, device="cuda")
    gdev.fill(L_d, 0, gen.ARR_L, gdev.DIST_SYM)
    gdev.fill(Lp_d, 0, gen.ARR_LPLUS, gdev.DIST_SYM)
    bufs = {}
    for lay in layouts:
        psi = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
        gdev.fill(psi, 0, gen.ARR_PSI, gdev.DIST_U01, LAYOUTS.index(lay), (D, G, Z))
        bufs[lay] = (psi, torch.empty(NM * G * Z, dtype=torch.float64, device="cuda"),
                     torch.empty(D * G * Z, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()

    # --- specialization (cold compiles, timed per key) -------------------------------------
    lib = P.lib()
    specs, handles, jit = {}, {}, {}
    for lay in layouts:
        for kname, kid in (("ltimes", P.SJ_LTIMES), ("lplustimes", P.SJ_LPLUSTIMES)):
            s = P.make_spec(layout=lay, Z=Z, G=G, D=D, NM=NM, **tile)
            t0 = time.perf_counter()
            h = P.sj_specialize(kid, s)
            wall = (time.perf_counter() - t0) * 1e3
            info = P.sj_handle_info(h)
            specs[(lay, kname)] = (kid, s)
            handles[(lay, kname)] = h
            jit[f"{kname}_{lay}"] = dict(wall_ms=round(wall, 1), emit_ms=round(info["emit_ms"], 3),
                                     compile_ms=round(info["compile_ms"], 1), load_ms=round(info["load_ms"], 2),
                                     vgprs=info["vgprs"], sgprs=info["sgprs"], scratch=info["scratch_bytes"],
                                     occupancy=info["occupancy"], lds=info["lds_bytes"], kernel=info["kernel_name"],
                                     variant=info["variant"], tile_n=info["tile_n"], tile_k=info["tile_k"],
                                     unroll=info["unroll"], block=info["block"])

    # Cache-hit latency of sj_specialize (through ctypes, so an upper bound).
    hout = ctypes.c_void_p()
    kid, s = specs[(layouts[0], "ltimes")]
    sref = ctypes.byref(s)
    n_hit = 20000
    t0 = time.perf_counter()
    for _ in range(n_hit):
        lib.sj_specialize(kid, sref, ctypes.byref(hout))
    hit_us = (time.perf_counter() - t0) / n_hit * 1e6

    arrs = {}
    for lay in layouts:
        psi, phi, out = bufs[lay]
        arrs[(lay, "ltimes")] = (ctypes.c_void_p * 3)(L_d.data_ptr(), psi.data_ptr(), phi.data_ptr())
        arrs[(lay, "lplustimes")] = (ctypes.c_void_p * 3)(Lp_d.data_ptr(), phi.data_ptr(), out.data_ptr())
    order = [(lay, k) for lay in layouts for k in ("ltimes", "lplustimes")]
    nbytes = algorithmic_bytes(Z, G, D, NM)

    def step(events=None):
        for key in order:
            kid, s = specs[key]
            rc = lib.sj_specialize(kid, ctypes.byref(s), ctypes.byref(hout))   # cache lookup (hit)
            if rc != 0:
                raise RuntimeError(P.sj_last_error())
            if events is not None:
                events[key][0].record(stream)
            rc = lib.sj_run(hout, arrs[key], 3, sptr)
            if events is not None:
                events[key][1].record(stream)
            if rc != 0:
                raise RuntimeError(P.sj_last_error())

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()

    evs = {key: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(a.steps)] for key in order}
    per_kernel = {key: [] for key in order}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step({key: evs[key][i] for key in order})
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for key in order:
        per_kernel[key] = [e0.elapsed_time(e1) for (e0, e1) in evs[key]]
    ms_per_step = wall * 1e3 / a.steps
    step_bytes = nbytes * len(order)
    value = step_bytes / (ms_per_step * 1e-3) / 1e9

    kern = {}
    for key in order:
        ms = statistics.median(per_kernel[key])
        kern[f"{key[1]}_{key[0]}"] = dict(us=round(ms * 1e3, 2), gbs=round(nbytes / (ms * 1e-3) / 1e9, 1),
                                           frac=round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    dom = max(order, key=lambda k: sum(per_kernel[k]))
    dom_ms = statistics.mean(per_kernel[dom])
    achieved = nbytes / (dom_ms * 1e-3) / 1e9

    # --- generic runtime-parameter kernels on the same buffers ----------------------------
    generic = {}
    if not a.no_generic:
        for lay in layouts:
            psi, phi, out = bufs[lay]
            for kname, kid, ptrs in (("ltimes", P.SJ_LTIMES, [L_d, psi, phi]),
                                     ("lplustimes", P.SJ_LPLUSTIMES, [Lp_d, phi, out])):
                gs = P.make_spec(layout=lay, Z=Z, G=G, D=D, NM=NM)
                for _ in range(2):
                    P.sj_generic_run(kid, ptrs, gs)
                ts = []
                for _ in range(max(3, a.steps // 2)):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    P.sj_generic_run(kid, ptrs, gs)
                    e1.record(stream)
                    ts.append((e0, e1))
                torch.cuda.synchronize()
                ms = statistics.median([x.elapsed_time(y) for x, y in ts])
                jit_us = kern[f"{kname}_{lay}"]["us"]
                generic[f"{kname}_{lay}"] = dict(us=round(ms * 1e3, 2), gbs=round(nbytes / (ms * 1e-3) / 1e9, 1),
                                                 jit_speedup=round(ms * 1e3 / jit_us, 3))

    # --- CPU oracle on a bounded sample of the same workload ------------------------------
    cpu = None
    if not a.no_cpu:
        import oracle
        threads = oracle.set_threads(0)
        L = gen.matrix_sym(0, gen.ARR_L, NM, D)
        Lp = gen.matrix_sym(0, gen.ARR_LPLUS, D, NM)
        zs = 2048
        done_bytes, spent = 0, 0.0
        lay_i = 0
        while spent < a.cpu_seconds and lay_i < 200:
            lay = layouts[lay_i % len(layouts)]
            z0 = (lay_i * zs) % Z
            cols = gen.psi_columns(0, D, G, Z, np.repeat(np.arange(G), zs), np.tile(np.arange(z0, z0 + zs), G))
            psi = gen.to_layout(cols.reshape(D, G, zs), lay)
            t0 = time.perf_counter()
            phi = oracle.ltimes(lay, zs, G, D, NM, L, psi)
            oracle.lplustimes(lay, zs, G, D, NM, Lp, phi)
            spent += time.perf_counter() - t0
            done_bytes += 2 * algorithmic_bytes(zs, G, D, NM)
            lay_i += 1
        cpu = dict(value=round(done_bytes / spent / 1e9, 3), unit="GB/s", cores=threads, kind="oracle",
                   sample=f"{lay_i} zone slabs of {zs} zones x G={G} (D={D}, NM={NM}), LTimes + LPlusTimes, "
                          f"nestings cycled {','.join(layouts)}; {spent:.1f} s of oracle time")

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (SplitMix64 counter generator, seed 0)",
        "config": {"workload": f"LTimes+LPlusTimes, six nestings chosen at run time, FP64, Z={Z} G={G} D={D} NM={NM}",
                   "layouts": layouts, "step": "per nesting: cache lookup + LTimes + LPlusTimes"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"{dom[1]}_{dom[0]}", "avg_us": round(dom_ms * 1e3, 2),
                     "bytes_per_launch": nbytes},
        "cpu_baseline": cpu,
        "kernels": kern,
        "generic": generic,
        "jit": jit,
        "cache_hit_us": round(hit_us, 3),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
