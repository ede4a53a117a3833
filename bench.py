#!/usr/bin/env python3
"""Benchmark: runtime-specialized LTimes / LPlusTimes on one MI355X.

Workload (default): all six nestings DGZ, DZG, GDZ, GZD, ZDG, ZGD chosen at run
time, FP64, Z = 32^3 = 32768 zones, G = 32 groups, D = 96 directions,
NM = 16 moments; psi ~ U[0,1), L and L+ ~ U[-1,1), seed 0 (counter-based
generator, values identical across layouts).  One step = for every nesting: the
specialization lookup (cache hit), LTimes psi -> phi, and LPlusTimes phi -> psi'.
Before the timed region the exhaustive tuner picks each nesting's and kernel's
specialization on the resident buffers (compiles in worker processes); the
same step with the library's default specializations is timed afterwards and
reported beside it (--no-tune skips the tuning).
All inputs are resident in HBM before the timed region; each array is 805 MB
or 134 MB, larger than the 256 MB last-level cache, so every step streams HBM.

Printed: one JSON line (metric, value = algorithmic GB/s of the whole step,
roofline of the dominant kernel from live HIP-event timing, the CPU oracle
baseline on a bounded sample, and the generic-kernel comparison).

Other workloads (--workload): batched (200,000 small products, HIP graph),
bf16 (split-BF16 LTimes at Z=262144 G=64 D=128 NM=64), picker (learned picker
against the exhaustive tuner), fused (LTimes then LPlusTimes in one pass),
values (weights compiled into the kernel), scattering (scattering source over
the six nestings), mass (tensor-product mass operator), copy (counter
calibration).  Each prints one JSON line of the same form.
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


# HBM bytes per launch measured with rocprofv3 (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, KiB per dispatch;
# both factors from a 1 GiB device copy), keyed by the SHA-1 of the emitted kernel source the counters
# were taken on: a kernel whose source has changed since reports traffic null.  The summaries with the
# commands are the trace-and-counter files of each workload under profiles/.
MEASURED_TRAFFIC = {
    # Z=32768 G=32 D=96 NM=16, the tuned specializations of the six nestings:
    "a72057a4a6e7a246a15903f0c958be7b7c6b376f": 940050043,  # sj_lplustimes_cols_mfma_zdg
    "2c7c9cdf86d4b19798fa6c15aa02847f433fd9de": 940673269,  # sj_lplustimes_direct_dgz
    "d29a392ebc2ce6e725c4dc61fcb1f8aa2e82d8b6": 940707834,  # sj_lplustimes_direct_dzg
    "65f93956b48e02a337a9396696699e9e7050d2e6": 940395639,  # sj_lplustimes_direct_gdz
    "6faf012bc4aa3239ccf5492f1f96d8dbd3205c72": 939731581,  # sj_lplustimes_rows_mfma_gzd
    "e92572674af57126b26f9a13a65126eeecfa5e3b": 939731197,  # sj_lplustimes_rows_mfma_zgd
    "aac6be0336c61377439e3d3e3634416ed9e6bae9": 939763195,  # sj_ltimes_direct_dgz
    "eab71f4174303315d32d91274d4ae3998ebd0aa5": 939762427,  # sj_ltimes_direct_dzg
    "11390ff2859129b666d598b3a0cfb489186094d5": 939998966,  # sj_ltimes_direct_gdz
    "75437275afe268eedc0d9369dd743e8d3ff4a576": 939734395,  # sj_ltimes_direct_zdg
    "b780dade1ba9509a8d304488318c03b07830cce1": 939694844,  # sj_ltimes_rows_mfma_lds_gzd
    "2c35009ddb2bddd0e9acd536270cc3e2c19c0777": 939694844,  # sj_ltimes_rows_mfma_lds_zgd
    # other winners of the tuning on other boxes:
    "096450941075a7b535ec0acdc4803e93fa480056": 940753013,  # sj_lplustimes_direct_dzg
    "5eefde36174a8c0697380a33840eb250c860eea7": 940605045,  # sj_lplustimes_direct_gdz
    "174c646463597e8495bac025d0588a78b135b42c": 939996918,  # sj_ltimes_direct_dgz
    "6c19c99e0e177b5af870248564a960d78c9da2a4": 939996278,  # sj_ltimes_direct_dzg
    # scattering (4 materials in zone regions, Z=32768 G=32 NM=16), default specializations:
    "5b273898027180bb79c395b49cf8c70e35f9030d": 270032989,  # sj_scattering_direct_gzd
    "f0a893edca371ae328b11107c4a596cd243f06c2": 270058588,  # sj_scattering_direct_zgd
    "72b818d409165b1caf6e7b882fec2e1d87c7090f": 269172848,  # sj_scattering_mfma_dgz
    "3b3f5766b2cce9423127a1ac1c61af4316f5e8a1": 270377301,  # sj_scattering_mfma_dzg
    "fa7a996b5cbceafbf17b0ee3785a13d0807319f2": 269172848,  # sj_scattering_mfma_gdz
    "f6d2343044c8bd43215bb791a188b82bc4755f23": 269865697,  # sj_scattering_mfma_zdg
    # mass operator (hex 500k elements, quad 2M elements, D=4 Q=6), default specializations:
    "760b6364988d89ff622be6ce3a7a360bcd546ea1": 1088243185,  # sj_mass_pa_pipe_2d_d4_q6
    "4d3e1c1b6b941ce74290c31c71bad133adf2f5e3": 1376579133,  # sj_mass_pa_pipe_3d_d4_q6
    # fused LTimes + LPlusTimes with phi written, default specializations:
    "b47cc03618f6aa006e91323d177850787fe8c381": 1678582454,  # sj_ltimes_lplus_direct_dgz
    "e9d19e8787d4e62dd0a5db2177e6f9099ae04d0c": 1678588662,  # sj_ltimes_lplus_direct_dzg
    "d47c27fd76a8582576f6f961a87ccc7b01705eeb": 1679043510,  # sj_ltimes_lplus_direct_gdz
    "1f9227015d887b2f9f4ce3d02f7ed6244aa22694": 1679022774,  # sj_ltimes_lplus_direct_zdg
    "7d67902c774d0d781d385cc6ee7e8c6d509e6e7c": 1678789171,  # sj_ltimes_lplus_rows_mfma_lds_gzd
    "5c68a857e356434db2f389ea39832cb23713d504": 1678762803,  # sj_ltimes_lplus_rows_mfma_lds_zgd
    # LTimes at Z=262144 G=64 D=128 NM=64 (BF16 forms: psi and phi FP32; FP64 forms):
    "1d98ee3ef25cf25ec41313284a3c5dd1789a6681": 12885323255,  # sj_ltimes_bf16_dgz
    "111efaeca57317b4febbd7e1e0bcd93abbe5ee20": 12961328927,  # sj_ltimes_bf16_rows_zgd
    "f6f07a961f0b57a5dea97134f5a51e5e4f71965b": 12885924913,  # sj_ltimes_bf16w_dgz
    "064caca9d342bd247e528f7049d4fd9123058c51": 12885361654,  # sj_ltimes_bf16x3_dgz
    "02608d4c7c058928c9748fb885a634bc6dbe4165": 12899945401,  # sj_ltimes_bf16x3_rows_zgd
    "11d9a11b89c49eb5977c1f64152ffa1996085ad5": 12885495542,  # sj_ltimes_bf16x3w_dgz
    # batched products, 200,000 instances n ~ U{3..16}, default specialization:
    "c3ba1c297bdc9d6ccad6fbee12c99a6e3f992468": 533975253,  # sj_bgemm_persistent
    # Z=32768 G=32 D=96 NM=16, another tuned set of the six nestings (the LDS-staged row LTimes with
    # two row tiles per wave, rotation and workgroups on contiguous XCD ranges):
    "caf4ba83110b0c9b595ccea83e82d168fa284f15": 940723317,  # sj_lplustimes_direct_dgz (read 134.7 MB, written 806.0 MB)
    "b5f2c3a8fd909fd198ad33fa9fcc6bf107e645fa": 940802293,  # sj_lplustimes_direct_dzg (read 134.7 MB, written 806.1 MB)
    "17fd69e3b29440e0f912deb3add2f6c1d8336777": 940737525,  # sj_lplustimes_direct_gdz (read 134.7 MB, written 806.0 MB)
    "57160d60ee27647a4376d637645887fbcdf2dc84": 940342136,  # sj_lplustimes_direct_zdg (read 134.6 MB, written 805.8 MB)
    "c9ee1470bfb94602eb0ea22725114c770abea167": 939964157,  # sj_lplustimes_rows_mfma_zgd (read 134.3 MB, written 805.6 MB)
    "4536cc7cb047bfe2cc8fe4196b61564ef4249a63": 939732731,  # sj_ltimes_direct_dgz (read 805.5 MB, written 134.2 MB)
    "133d138961c05fb37623878b4f19d58e5f256ae1": 939995126,  # sj_ltimes_direct_dzg (read 805.8 MB, written 134.2 MB)
    "f9e011450da5ffd5c729f1fc92560b93116f25d1": 939694844,  # sj_ltimes_rows_mfma_lds_gzd (read 805.5 MB, written 134.2 MB)
    "39f562d0cb6361bc8681a427185ee496c7bbf708": 939694844,  # sj_ltimes_rows_mfma_lds_zgd (read 805.5 MB, written 134.2 MB)
}


# Matrix-core busy fraction measured with rocprofv3 (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE / 8
# x 1024 SIMDs), keyed like MEASURED_TRAFFIC; the summary with the commands is
# profiles/mfma_busy_moments_bf16_bgemm_counters.md.
MEASURED_MFMA_BUSY = {
    # Z=32768 G=32 D=96 NM=16 (FP64 matrix cores)
    "a72057a4a6e7a246a15903f0c958be7b7c6b376f": 0.219,  # sj_lplustimes_cols_mfma_zdg
    "6faf012bc4aa3239ccf5492f1f96d8dbd3205c72": 0.181,  # sj_lplustimes_rows_mfma_gzd
    "e92572674af57126b26f9a13a65126eeecfa5e3b": 0.182,  # sj_lplustimes_rows_mfma_zgd
    "b780dade1ba9509a8d304488318c03b07830cce1": 0.261,  # sj_ltimes_rows_mfma_lds_gzd
    "2c35009ddb2bddd0e9acd536270cc3e2c19c0777": 0.260,  # sj_ltimes_rows_mfma_lds_zgd
    # the same shape, the second tuned set (two row tiles per wave, rotation, contiguous XCD ranges)
    "f9e011450da5ffd5c729f1fc92560b93116f25d1": 0.262,  # sj_ltimes_rows_mfma_lds_gzd
    "39f562d0cb6361bc8681a427185ee496c7bbf708": 0.259,  # sj_ltimes_rows_mfma_lds_zgd
    "c9ee1470bfb94602eb0ea22725114c770abea167": 0.222,  # sj_lplustimes_rows_mfma_zgd
    # Z=262144 G=64 D=128 NM=64: FP64 column kernel, BF16 forms
    "1d98ee3ef25cf25ec41313284a3c5dd1789a6681": 0.037,  # sj_ltimes_bf16_dgz
    "111efaeca57317b4febbd7e1e0bcd93abbe5ee20": 0.047,  # sj_ltimes_bf16_rows_zgd
    "f6f07a961f0b57a5dea97134f5a51e5e4f71965b": 0.048,  # sj_ltimes_bf16w_dgz
    "064caca9d342bd247e528f7049d4fd9123058c51": 0.129,  # sj_ltimes_bf16x3_dgz
    "02608d4c7c058928c9748fb885a634bc6dbe4165": 0.162,  # sj_ltimes_bf16x3_rows_zgd
    "11d9a11b89c49eb5977c1f64152ffa1996085ad5": 0.175,  # sj_ltimes_bf16x3w_dgz
    "60467b2e08b71a9f23cd2cf2872db0e82932347b": 0.766,  # sj_ltimes_cols_mfma_dgz
    # batched products, 200,000 instances n ~ U{3..16}
    "c3ba1c297bdc9d6ccad6fbee12c99a6e3f992468": 0.169,  # sj_bgemm_persistent
}


def mfma_evidence(P, kernel, spec, flops, us, peak_tflops):
    """Matrix-core use of a launch: the counter-measured busy fraction (None when the counters were
    not taken on this exact kernel source) and the algorithmic flop rate against the dtype's peak."""
    tf = flops / (us * 1e-6) / 1e12
    return {"busy_frac": MEASURED_MFMA_BUSY.get(source_sha1(P, kernel, spec)),
            "achieved_tflops": round(tf, 2), "peak_tflops": peak_tflops, "frac_of_peak": round(tf / peak_tflops, 4)}


def source_sha1(P, kernel, spec):
    """SHA-1 of the emitted source of a specialization: names the exact kernel that counters were taken on."""
    import hashlib
    return hashlib.sha1(P.sj_emit_source(kernel, spec).encode()).hexdigest()


def measured_traffic(P, kernel, spec):
    """HBM bytes per launch from the counters if they were taken on this exact kernel source, else None."""
    return MEASURED_TRAFFIC.get(source_sha1(P, kernel, spec))


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
    ap.add_argument("--layouts", default="", help="comma-separated nestings (default: all six, in the order of LAYOUTS)")
    ap.add_argument("--no-generic", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the CPU baseline sample")
    ap.add_argument("--tile", default="", help="override tile params, e.g. 'tile_n=2,unroll=8,block=256'")
    ap.add_argument("--no-tune", action="store_true",
                    help="moments: time the default specializations only (no exhaustive tuning first)")
    ap.add_argument("--out-dir", default="bench_out",
                    help="directory for the tuning results (tuned_moments.json) and the picker's data")
    ap.add_argument("--tuned-json", default="",
                    help="moments: take the tuned specializations from this file (written by an earlier run to "
                         "<out-dir>/tuned_moments.json) instead of tuning")
    ap.add_argument("--in-step-sweep", default="",
                    help="moments: comma-separated NESTING:kernel items (e.g. GZD:ltimes); every tuner candidate of "
                         "each, with ordinary and with nontemporal stores, is timed inside the whole step")
    ap.add_argument("--picker-part", default="all", choices=("all", "collect", "evaluate"))
    ap.add_argument("--picker-slice", default="", help="held-out shapes lo:hi, or train (the training timings), for --picker-part collect")
    ap.add_argument("--picker-data", default="", help="comma-separated collect outputs for --picker-part evaluate")
    ap.add_argument("--workload", default="moments", choices=("moments", "batched", "bf16", "picker", "copy", "fused", "values", "scattering", "mass",
                             "small"),
                    help="moments: six nestings FP64 (default); batched: 200k small products; "
                         "bf16: LTimes Z=262144 G=64 D=128 NM=64 in BF16/BF16x3/FP64")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU: this library has no multi-GPU path (asked for --gpus {a.gpus}); "
              "the contractions are independent per (g, z) column, so N GPUs would each run the one-GPU kernel "
              "on a zone shard.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1904_08555_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.sj_init(0)
    if a.workload == "batched":
        return bench_batched(a)
    if a.workload == "bf16":
        return bench_bf16(a)
    if a.workload == "picker":
        return bench_picker(a)
    if a.workload == "copy":
        return bench_copy(a)
    if a.workload == "fused":
        return bench_fused(a)
    if a.workload == "values":
        return bench_values(a)
    if a.workload == "scattering":
        return bench_scattering(a)
    if a.workload == "mass":
        return bench_mass(a)
    if a.workload == "small":
        return bench_small(a)
    return bench_moments(a)


def bench_moments(a):
    import numpy as np
    import torch

    import paper_1904_08555_amd as P
    import sj_inputs as gen
    from sj_inputs import device as gdev

    Z, G, D, NM = a.Z, a.G, a.D, a.NM
    layouts = [x for x in a.layouts.split(",") if x] or list(LAYOUTS)
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
    default_specs = {}
    for lay in layouts:
        for kname, kid in (("ltimes", P.SJ_LTIMES), ("lplustimes", P.SJ_LPLUSTIMES)):
            default_specs[(lay, kname)] = (kid, P.make_spec(layout=lay, Z=Z, G=G, D=D, NM=NM, **tile))

    # --- exhaustive tuning on the resident buffers (compiles in worker processes) ----------
    tuned, tune_s, ranked = {}, None, {}
    if a.tuned_json:
        with open(a.tuned_json) as f:
            for k, v in json.load(f).items():
                kname, lay = k.split("_")
                if lay in layouts:
                    tuned[(lay, kname)] = v
    elif not a.no_tune and not tile:
        from paper_1904_08555_amd import tune
        from paper_1904_08555_amd.farm import CompileFarm
        t0 = time.perf_counter()
        with CompileFarm(12) as farm:
            for lay in layouts:
                psi, phi, out = bufs[lay]
                for kname, kid, ptrs in (("ltimes", P.SJ_LTIMES, [L_d, psi, phi]),
                                         ("lplustimes", P.SJ_LPLUSTIMES, [Lp_d, phi, out])):
                    r = tune.tune_exhaustive(kid, lay, Z, G, D, NM, ptrs, reps=10, warmup=2, farm=farm)
                    tuned[(lay, kname)] = r["best"]
                    ranked[(lay, kname)] = [c for c, _, _ in sorted(r["results"], key=lambda x: x[1])[:3]]
                    print(f"tuned {kname} {lay}: {r['best']} {r['best_ms'] * 1e3:.1f} us "
                          f"({len(r['results'])} candidates)", file=sys.stderr, flush=True)
        tune_s = time.perf_counter() - t0
        os.makedirs(os.path.join(ROOT, a.out_dir), exist_ok=True)
        with open(os.path.join(ROOT, a.out_dir, "tuned_moments.json"), "w") as f:
            json.dump({f"{k[1]}_{k[0]}": v for k, v in tuned.items()}, f)
    for lay in layouts:
        for kname, kid in (("ltimes", P.SJ_LTIMES), ("lplustimes", P.SJ_LPLUSTIMES)):
            s = P.make_spec(layout=lay, Z=Z, G=G, D=D, NM=NM, **(tuned.get((lay, kname)) or tile))
            h = P.sj_specialize(kid, s)
            specs[(lay, kname)] = (kid, s)
            handles[(lay, kname)] = h

    # Cache-hit latency of sj_specialize (through ctypes, so an upper bound).
    hout = ctypes.c_void_p()
    kid, s = specs[(layouts[0], "ltimes")]
    sref = ctypes.byref(s)
    n_hit = 20000
    t0 = time.perf_counter()
    for _ in range(n_hit):
        lib.sj_specialize(kid, sref, ctypes.byref(hout))
    hit_us = (time.perf_counter() - t0) / n_hit * 1e6

    # Native hit latency from 1 and 8 threads (a child process running the C ABI
    # in a loop; the interpreter's own per-call cost is excluded).
    import subprocess
    native = {}
    exe = os.path.join(ROOT, "paper_1904_08555_amd", "sj_lookup_bench")
    for nt in (1, 8):
        r = subprocess.run([exe, str(nt), "200000", "0"], capture_output=True, text=True, timeout=120)
        native[nt] = json.loads(r.stdout)["ns_per_hit_median"] if r.returncode == 0 else None
    arrs = {}
    for lay in layouts:
        psi, phi, out = bufs[lay]
        arrs[(lay, "ltimes")] = (ctypes.c_void_p * 3)(L_d.data_ptr(), psi.data_ptr(), phi.data_ptr())
        arrs[(lay, "lplustimes")] = (ctypes.c_void_p * 3)(Lp_d.data_ptr(), phi.data_ptr(), out.data_ptr())
    order = [(lay, k) for lay in layouts for k in ("ltimes", "lplustimes")]
    nbytes = algorithmic_bytes(Z, G, D, NM)

    def step(events=None, table=specs):
        for key in order:
            kid, s = table[key]
            rc = lib.sj_specialize(kid, ctypes.byref(s), ctypes.byref(hout))   # cache lookup (hit)
            if rc != 0:
                raise RuntimeError(P.sj_last_error())
            if events is not None and key in events:
                events[key][0].record(stream)
            rc = lib.sj_run(hout, arrs[key], 3, sptr)
            if events is not None and key in events:
                events[key][1].record(stream)
            if rc != 0:
                raise RuntimeError(P.sj_last_error())

    # In-step refinement of the tuned choices: a kernel's speed depends on the one
    # before it (the previous LPlusTimes' writes are still draining when the next
    # LTimes starts; LPlusTimes reads the phi that LTimes has just written), which
    # the isolated tuning cannot see.  Each kernel in turn tries its three best
    # isolated candidates, the library default and, for LTimes, the best and the
    # default with ordinary stores, inside the whole step, and keeps the one with
    # the lowest median step time; two passes over the twelve kernels.
    refined = 0
    if ranked:
        def step_ms(reps=9):
            for _ in range(2):
                step()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                step()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            return statistics.median(ts) * 1e3
        def choices(key):
            out = list(ranked.get(key, [])) + [{}]
            if key[1] == "ltimes":
                # phi (134 MB) written with ordinary stores can stay in the last-level
                # cache for the LPlusTimes that reads it next
                for c in (ranked[key][0] if ranked.get(key) else None, {}):
                    if c is not None:
                        c2 = dict(c)
                        c2["flags"] = (c2.get("flags", 0) & ~P.SJ_FLAG_STORES_NONTEMPORAL) | P.SJ_FLAG_STORES_CACHED
                        out.append(c2)
            return out
        for _ in range(2):   # two passes: a choice can change which choice is best for its neighbour
            for key in order:
                kid, lay = specs[key][0], key[0]
                best_spec, best_t = specs[key], step_ms()
                for c in choices(key):
                    if c == tuned.get(key):
                        continue
                    specs[key] = (kid, P.make_spec(layout=lay, Z=Z, G=G, D=D, NM=NM, **c))
                    t = step_ms()
                    if t < best_t:
                        best_spec, best_t = specs[key], t
                        tuned[key] = c
                        refined += 1
                specs[key] = best_spec
        with open(os.path.join(ROOT, a.out_dir, "tuned_moments.json"), "w") as f:
            json.dump({f"{k[1]}_{k[0]}": v for k, v in tuned.items()}, f)

    # Optional: every candidate of the named kernels inside the whole step (the other kernels at
    # their chosen specializations): the kernel's own median time and the step's
    sweep = {}
    if a.in_step_sweep:
        from paper_1904_08555_amd import tune
        for item in a.in_step_sweep.split(","):
            lay, kname = item.split(":")
            key = (lay, kname)
            kid, keep = specs[key][0], specs[key]
            stores = (P.SJ_FLAG_STORES_CACHED, P.SJ_FLAG_STORES_NONTEMPORAL)
            cands = [dict(c, flags=(c.get("flags", 0) | fl)) for c in tune.candidates(kid, lay, Z, G, D, NM)
                     for fl in stores]
            base = dict(layout=lay, Z=Z, G=G, D=D, NM=NM)
            rows = []
            for c, h, err in tune.compile_all(kid, base, tune.distinct(kid, base, cands)):
                if h is None:
                    continue
                specs[key] = (kid, P.make_spec(**base, **c))
                for _ in range(2):
                    step()
                kev, sev = [], []
                for _ in range(9):
                    e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    s0.record(stream)
                    step({key: e})
                    s1.record(stream)
                    kev.append(e)
                    sev.append((s0, s1))
                torch.cuda.synchronize()
                rows.append(dict(spec=c, kernel=P.sj_handle_info(h)["kernel_name"],
                                 kernel_us=round(statistics.median(x.elapsed_time(y) for x, y in kev) * 1e3, 1),
                                 step_us=round(statistics.median(x.elapsed_time(y) for x, y in sev) * 1e3, 1)))
            specs[key] = keep
            sweep[item] = sorted(rows, key=lambda r: r["step_us"])

    # the specializations the timed steps use (after any refinement)
    for key in order:
        kid, s = specs[key]
        info = P.sj_handle_info(P.sj_specialize(kid, s))
        jit[f"{key[1]}_{key[0]}"] = dict(kernel=info["kernel_name"], variant=info["variant"], tile_n=info["tile_n"],
                                         tile_k=info["tile_k"], unroll=info["unroll"], block=info["block"],
                                         vgprs=info["vgprs"], scratch=info["scratch_bytes"],
                                         occupancy=info["occupancy"], lds=info["lds_bytes"],
                                         src_sha1=source_sha1(P, kid, s), traffic=measured_traffic(P, kid, s),
                                         mfma_busy=MEASURED_MFMA_BUSY.get(source_sha1(P, kid, s)))
    # cold specialization cost: ten keys never compiled before, in this process
    cold = []
    for i in range(10):
        kid_c = P.SJ_LTIMES if i % 2 == 0 else P.SJ_LPLUSTIMES
        t0 = time.perf_counter()
        hc = P.sj_specialize(kid_c, layout=layouts[i % len(layouts)], Z=Z + 64 * (i + 1), G=G, D=D, NM=NM)
        wall = (time.perf_counter() - t0) * 1e3
        ic = P.sj_handle_info(hc)
        cold.append((wall, ic["emit_ms"], ic["compile_ms"], ic["load_ms"]))
    jit_cold = {name: round(statistics.median(x[j] for x in cold), 3)
                for j, name in enumerate(("wall_ms", "emit_ms", "compile_ms", "load_ms"))}

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
        sd = statistics.stdev(per_kernel[key]) if len(per_kernel[key]) > 1 else 0.0
        kern[f"{key[1]}_{key[0]}"] = dict(us=round(ms * 1e3, 2), std_us=round(sd * 1e3, 2),
                                           gbs=round(nbytes / (ms * 1e-3) / 1e9, 1),
                                           frac=round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    # the measured device-copy rate (1 GiB read + 1 GiB written), the practical ceiling beside the nominal peak
    csrc = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
    cdst = torch.empty_like(csrc)
    cmed, _ = time_launches(lambda: cdst.copy_(csrc), 10, torch.cuda.current_stream())
    copy_gbs = 2 * (1 << 30) / (cmed * 1e-3) / 1e9
    del csrc, cdst
    # the same step with the default (untuned) specializations (skipped when the
    # tuned choices come from a file, as in a profiled run)
    default_value = None
    if tuned and not a.tuned_json:
        for _ in range(a.warmup):
            step(table=default_specs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            step(table=default_specs)
        torch.cuda.synchronize()
        default_value = step_bytes / ((time.perf_counter() - t0) / a.steps) / 1e9

    # every kernel alone with a 1 GiB scratch read before each launch: nothing of its operands in the
    # last-level cache (in the step, LPlusTimes may read part of the phi that LTimes has just written
    # from the 256 MB last-level cache, so its in-step figures are cache-assisted)
    scratch = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
    for key in order:
        kid_k, s_k = specs[key]
        h_k = P.sj_specialize(kid_k, s_k)
        ptrs_k = arrs[key]
        ms_k, _ = time_launches(lambda: lib.sj_run(h_k.ptr, ptrs_k, 3, sptr), max(5, a.steps // 2), stream, scratch)
        kern[f"{key[1]}_{key[0]}"].update(isolated_hbm_us=round(ms_k * 1e3, 2),
                                          isolated_hbm_frac=round(nbytes / (ms_k * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    del scratch
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
                res_g = {}
                # one kernel for every nesting, and the kernel compiled for this nesting (sizes at run time)
                for mode, fl in (("", 0), ("per_layout_", P.SJ_FLAG_GENERIC_PER_LAYOUT)):
                    gs = P.make_spec(layout=lay, Z=Z, G=G, D=D, NM=NM, flags=fl)
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
                    res_g.update({f"{mode}us": round(ms * 1e3, 2), f"{mode}gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                                  f"{mode}jit_speedup": round(ms * 1e3 / jit_us, 3)})
                generic[f"{kname}_{lay}"] = res_g

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
        while spent < a.cpu_seconds and lay_i < 5000:
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
        # the same oracle on one thread, a few slabs (about 3 s)
        oracle.set_threads(1)
        b1, s1, k = 0, 0.0, 0
        while s1 < min(3.0, a.cpu_seconds) and k < 500:
            lay = layouts[k % len(layouts)]
            cols = gen.psi_columns(0, D, G, Z, np.repeat(np.arange(G), zs), np.tile(np.arange(zs), G))
            psi = gen.to_layout(cols.reshape(D, G, zs), lay)
            t0 = time.perf_counter()
            phi = oracle.ltimes(lay, zs, G, D, NM, L, psi)
            oracle.lplustimes(lay, zs, G, D, NM, Lp, phi)
            s1 += time.perf_counter() - t0
            b1 += 2 * algorithmic_bytes(zs, G, D, NM)
            k += 1
        oracle.set_threads(threads)
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        cpu.update(single_thread_value=round(b1 / s1 / 1e9, 3), single_thread_sample=f"{k} slabs, {s1:.1f} s",
                   host_cpu=model, host_logical_cpus=os.cpu_count())

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
                   "layouts": layouts, "step": "per nesting: cache lookup + LTimes + LPlusTimes",
                   "specialization": ("chosen per nesting and kernel by the exhaustive tuner before the timed region"
                                      if tuned else "library defaults")},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(P, *specs[dom]),
                     "kernel": f"{dom[1]}_{dom[0]}", "avg_us": round(dom_ms * 1e3, 2),
                     "bytes_per_launch": nbytes, "measured_copy_gbs": round(copy_gbs, 1),
                     "frac_of_measured_copy": round(achieved / copy_gbs, 4),
                     "mfma": mfma_evidence(P, *specs[dom], 2 * D * NM * G * Z, dom_ms * 1e3, 78.6)},
        "step_frac_of_measured_copy": round(value / copy_gbs, 4),
        "value_note": ("effective rate of the step: algorithmic bytes / step time; LPlusTimes may read part of phi "
                       "from the last-level cache right after LTimes writes it, so per-kernel in-step figures of "
                       "LPlusTimes are cache-assisted; isolated_hbm_* are each kernel alone with the cache flushed"),
        "cpu_baseline": cpu,
        "kernels": kern,
        "generic": generic,
        "jit": jit,
        "jit_cold_median_of_10_keys": jit_cold,
        "cache_hit_us_ctypes": round(hit_us, 3),
        "cache_hit_ns_native": native[1],
        "cache_hit_ns_native_8_threads": native[8],
        "tuned": {f"{k[1]}_{k[0]}": v for k, v in tuned.items()},
        "tune_s": None if tune_s is None else round(tune_s, 1),
        "refined_in_step": refined,
        "in_step_sweep": sweep or None,
        "value_default_specializations": None if default_value is None else round(default_value, 1),
    }
    print(json.dumps(line), flush=True)


def time_launches(fn, reps, stream, flush=None, warmup=0):
    """Median and mean duration (ms) of `reps` launches of fn, each bracketed by
    events; with ``flush`` (a float64 device tensor) the tensor is read in full
    before every launch, outside the bracket, so the launch finds nothing of
    its operands in L2 or the last-level cache.  Reading, not writing: a
    written scratch buffer leaves dirty lines whose write-back would fall into
    the timed launch (measured: LPlusTimes DGZ 202 us after a 1 GiB write,
    177 us after a 1 GiB read).  ``warmup`` untimed launches come first."""
    import torch
    for _ in range(warmup):
        fn()
    evs = []
    for _ in range(reps):
        if flush is not None:
            flush.sum()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    ts = [x.elapsed_time(y) for x, y in evs]
    return statistics.median(ts), statistics.mean(ts)


def bench_batched(a):
    """200,000 products C_i = A_i B_i, n_i ~ U{3..16}, A, B ~ N(0,1), FP64.
    One step = one replay of the HIP graph holding the persistent launch."""
    import numpy as np
    import torch

    import paper_1904_08555_amd as P
    import sj_inputs as gen

    count = 200000
    n = gen.batch_sizes(0, count)
    off = gen.batch_offsets(n)
    total = int(off[-1])
    A_d = torch.from_numpy(gen.batch_normal(0, gen.ARR_A, total)).cuda()
    B_d = torch.from_numpy(gen.batch_normal(0, gen.ARR_B, total)).cuda()
    C_d = torch.empty(total, dtype=torch.float64, device="cuda")
    flush = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")   # read to evict L2 and the LLC
    tile = {}
    for kv in filter(None, a.tile.split(",")):
        k, v = kv.split("=")
        tile[k] = int(v)
    tuned_by, tune_s, n_tuned = "library default", None, 0
    if not tile and not a.no_tune:
        # the tiles come from the exhaustive tuner, timed on this batch (scratch read before each launch)
        from paper_1904_08555_amd import tune
        from paper_1904_08555_amd.farm import CompileFarm
        t0 = time.perf_counter()
        with CompileFarm(12) as farm:
            r = tune.tune_bgemm(n, A_d, B_d, C_d, reps=5, warmup=1, flush=flush, farm=farm)
        tune_s = time.perf_counter() - t0
        tile, tuned_by, n_tuned = dict(r["best"]), "exhaustive tuner (tune.tune_bgemm)", len(r["results"])
        print(f"tuned batched products: {tile} {r['best_ms'] * 1e3:.1f} us ({n_tuned} candidates)",
              file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    h = P.sj_specialize(P.SJ_BGEMM, **tile)
    jit_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    plan = P.sj_batch_plan(h, n)
    plan_ms = (time.perf_counter() - t0) * 1e3
    P.sj_batch_graph_capture(plan, A_d, B_d, C_d)
    stream = torch.cuda.current_stream()
    nbytes = 3 * total * 8
    flops = 2 * int(np.sum(n.astype(np.int64) ** 3))
    for _ in range(a.warmup):
        P.sj_batch_graph_launch(plan)
    torch.cuda.synchronize()

    def flushed(fn, reps):
        """Per-launch event times (ms) and host wall time (s), with a 1 GiB
        scratch read before every launch (the working set fits the LLC otherwise).
        The launch is enqueued behind the scratch read, so the events bracket the
        GPU's work and not the host's submission latency; the wall time keeps it."""
        per, wall = [], 0.0
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            flush.sum()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            per.append(e0.elapsed_time(e1))
        return per, wall

    per, t_total = flushed(lambda: P.sj_batch_graph_launch(plan), a.steps)
    med = statistics.median(per)
    # the kernel's own duration: events around direct launches (a graph replay adds launch latency)
    run_per, _ = flushed(lambda: P.sj_batch_run(plan, A_d, B_d, C_d), a.steps)
    mean = statistics.mean(run_per)
    n_dev, off_dev, _ = P.sj_batch_plan_arrays(plan)
    gspec = P.make_spec(count=count)

    def generic():
        P.sj_generic_run(P.SJ_BGEMM, [n_dev, off_dev, A_d, B_d, C_d], gspec)
    generic()
    gper, _ = flushed(generic, max(3, a.steps // 2))
    gmed = statistics.median(gper)
    # the generic kernel captured in a graph of its own, so that graph replay meets graph replay
    # (a replay costs the same fixed time over a direct launch whatever kernel it holds); its
    # output is checked bit for bit against the direct launch's before it is timed
    torch.cuda.synchronize()
    c_direct = C_d.clone()
    ggraph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(ggraph):
        generic()
    for _ in range(2):
        C_d.zero_()
        ggraph.replay()
        torch.cuda.synchronize()
        if not torch.equal(C_d, c_direct):
            raise RuntimeError("the graph-captured generic batched product differs from its direct launch")
    ggper, _ = flushed(ggraph.replay, max(3, a.steps // 2))
    ggmed = statistics.median(ggper)
    del ggraph, c_direct
    info = P.sj_handle_info(h)
    # the device-copy rate (512 MB read and written, the scratch read before each copy), the practical
    # ceiling of a stream that reads and writes
    csrc = torch.ones(total, dtype=torch.float64, device="cuda")
    cdst = torch.empty_like(csrc)
    cmed, _ = time_launches(lambda: cdst.copy_(csrc), max(5, a.steps // 2), stream, flush, warmup=2)
    copy_gbs = 2 * total * 8 / (cmed * 1e-3) / 1e9
    del csrc, cdst
    line = {
        "metric": "batched small products GB/s (persistent per-class graph launch vs per-instance generic)",
        "value": round(nbytes / (med * 1e-3) / 1e9, 1), "unit": "GB/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(med, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (SplitMix64, seed 0)",
        "config": {"workload": "200000 products, n ~ U{3..16}, A,B ~ N(0,1), FP64, packed row-major",
                   "total_elements": total, "flops": flops},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / (mean * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(nbytes / (mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(P, P.SJ_BGEMM, P.make_spec(**tile)),
                     "kernel": info["kernel_name"], "avg_us": round(mean * 1e3, 2), "bytes_per_launch": nbytes,
                     "src_sha1": source_sha1(P, P.SJ_BGEMM, P.make_spec(**tile)),
                     "mfma": mfma_evidence(P, P.SJ_BGEMM, P.make_spec(**tile), flops, mean * 1e3, 78.6)},
        "graph_us_median": round(med * 1e3, 2), "direct_launch_us_median": round(statistics.median(run_per) * 1e3, 2),
        "host_wall_ms_per_step_with_scratch_write": round(t_total * 1e3 / a.steps, 4),
        "generic_us": round(gmed * 1e3, 2),
        "speedup_vs_generic": round(gmed / med, 3),
        "direct_launch_speedup_vs_generic": round(gmed / statistics.median(run_per), 3),
        "generic_graph_us": round(ggmed * 1e3, 2),
        "speedup_vs_generic_graph": round(ggmed / med, 3),
        "measured_copy_gbs": round(copy_gbs, 1),
        "direct_launch_frac_of_measured_copy": round(nbytes / (statistics.median(run_per) * 1e-3) / 1e9 / copy_gbs, 4),
        "jit_ms": round(jit_ms, 1), "plan_ms": round(plan_ms, 1),
        "tiles": tile, "tiles_from": tuned_by, "tuned_candidates": n_tuned,
        "tune_s": None if tune_s is None else round(tune_s, 1),
        "kernel_info": {k: info[k] for k in ("vgprs", "sgprs", "occupancy", "lds_bytes", "scratch_bytes", "block",
                                             "variant", "tile_n", "unroll")},
    }
    P.sj_plan_destroy(plan)
    print(json.dumps(line), flush=True)


def bench_bf16(a):
    """LTimes, DGZ, Z=262144 G=64 D=128 NM=64: BF16 (psi FP32 in, phi FP32 out),
    compensated BF16x3, and the FP64 path on the same values; also both BF16
    modes with D innermost (ZGD, the row form)."""
    import torch

    import paper_1904_08555_amd as P
    import sj_inputs as gen
    from sj_inputs import device as gdev

    Z, G, D, NM = 262144, 64, 128, 64
    L_d = torch.empty(NM * D, dtype=torch.float64, device="cuda")
    gdev.fill(L_d, 0, gen.ARR_L, gdev.DIST_SYM)
    psi32 = torch.empty(D * G * Z, dtype=torch.float32, device="cuda")
    gdev.fill(psi32, 0, gen.ARR_PSI, gdev.DIST_U01_24, 0, (D, G, Z))
    phi32 = torch.empty(NM * G * Z, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    b32 = (D + NM) * G * Z * 4 + NM * D * 8
    # default (wide, four columns per lane) and the one-column-per-lane form
    for name, dt, cols in (("bf16", P.SJ_BF16, 0), ("bf16x3", P.SJ_BF16X3, 0),
                           ("bf16_narrow", P.SJ_BF16, 1), ("bf16x3_narrow", P.SJ_BF16X3, 1)):
        spec = P.make_spec(layout="DGZ", Z=Z, G=G, D=D, NM=NM, dtype=dt, tile_n=cols)
        h = P.sj_specialize(P.SJ_LTIMES, spec)
        t = P.sj_time_run(h, [L_d, psi32, phi32], warmup=a.warmup, reps=a.steps)
        ms = statistics.median(t)
        info = P.sj_handle_info(h)
        res[name] = dict(ms=round(ms, 4), gbs=round(b32 / (ms * 1e-3) / 1e9, 1),
                         frac=round(b32 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), kernel=info["kernel_name"],
                         vgprs=info["vgprs"], agprs=info["agprs"], occupancy=info["occupancy"],
                         src_sha1=source_sha1(P, P.SJ_LTIMES, spec), traffic=measured_traffic(P, P.SJ_LTIMES, spec),
                         mfma=mfma_evidence(P, P.SJ_LTIMES, spec, (3 if dt == P.SJ_BF16X3 else 1) * 2 * D * NM * G * Z,
                                            ms * 1e3, 2500.0))
    # D innermost (ZGD): the row form, on the same logical values stored in that nesting
    gdev.fill(psi32, 0, gen.ARR_PSI, gdev.DIST_U01_24, LAYOUTS.index("ZGD"), (D, G, Z))
    for name, dt in (("bf16_zgd", P.SJ_BF16), ("bf16x3_zgd", P.SJ_BF16X3)):
        spec = P.make_spec(layout="ZGD", Z=Z, G=G, D=D, NM=NM, dtype=dt)
        h = P.sj_specialize(P.SJ_LTIMES, spec)
        t = P.sj_time_run(h, [L_d, psi32, phi32], warmup=a.warmup, reps=a.steps)
        ms = statistics.median(t)
        info = P.sj_handle_info(h)
        res[name] = dict(ms=round(ms, 4), gbs=round(b32 / (ms * 1e-3) / 1e9, 1),
                         frac=round(b32 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), kernel=info["kernel_name"],
                         vgprs=info["vgprs"], agprs=info["agprs"], occupancy=info["occupancy"],
                         src_sha1=source_sha1(P, P.SJ_LTIMES, spec), traffic=measured_traffic(P, P.SJ_LTIMES, spec),
                         mfma=mfma_evidence(P, P.SJ_LTIMES, spec, (3 if dt == P.SJ_BF16X3 else 1) * 2 * D * NM * G * Z,
                                            ms * 1e3, 2500.0))
    gdev.fill(psi32, 0, gen.ARR_PSI, gdev.DIST_U01_24, 0, (D, G, Z))
    del phi32
    psi64 = psi32.to(torch.float64)
    del psi32
    phi64 = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
    b64 = (D + NM) * G * Z * 8 + NM * D * 8
    flops = 2 * D * NM * G * Z
    # FP64: vector FMAs (DIRECT) and the FP64 matrix-core column kernel
    for name, var in (("f64", P.SJ_VAR_DIRECT), ("f64_mfma", P.SJ_VAR_MFMA)):
        spec = P.make_spec(layout="DGZ", Z=Z, G=G, D=D, NM=NM, variant=var)
        h = P.sj_specialize(P.SJ_LTIMES, spec)
        t = P.sj_time_run(h, [L_d, psi64, phi64], warmup=a.warmup, reps=a.steps)
        ms = statistics.median(t)
        info = P.sj_handle_info(h)
        res[name] = dict(ms=round(ms, 4), gbs=round(b64 / (ms * 1e-3) / 1e9, 1), kernel=info["kernel_name"],
                         tflops=round(flops / (ms * 1e-3) / 1e12, 2),
                         frac_fp64_peak=round(flops / (ms * 1e-3) / 78.6e12, 4),
                         mfma=mfma_evidence(P, P.SJ_LTIMES, spec, flops, ms * 1e3, 78.6))
    best = res["bf16x3"]
    line = {
        "metric": "LTimes BF16 (split-compensated) GB/s at Z=262144 G=64 D=128 NM=64",
        "value": best["gbs"], "unit": "GB/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": best["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3 (fp32 accumulate)", "data": "synthetic (SplitMix64, seed 0)",
        "config": {"workload": "LTimes DGZ Z=262144 G=64 D=128 NM=64, psi FP32 in, phi FP32 out"},
        "roofline": {"bound": "hbm", "achieved": best["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": best["frac"], "traffic": best["traffic"], "kernel": best["kernel"], "bytes_per_launch": b32,
                     "mfma": best["mfma"]},
        "modes": res,
    }
    print(json.dumps(line), flush=True)


def bench_values(a):
    """LTimes and LPlusTimes with the weights compiled into the kernel (value
    specialization) against the same DIRECT kernel reading them at run time
    (same tiles, order 1) and against the library default, DGZ, FP64,
    Z=32768 G=32 D=96 NM=16.  Weights: the dense matrices of the main workload;
    the same with every other direction's coefficients zero (moments of half
    the directions); one-hot (each moment takes one direction).  value = GB/s of
    the dense value-specialized LTimes (algorithmic bytes / median time)."""
    import numpy as np
    import torch

    import paper_1904_08555_amd as P
    import sj_inputs as gen
    from sj_inputs import device as gdev

    Z, G, D, NM = a.Z, a.G, a.D, a.NM
    lay = "DGZ"
    stream = torch.cuda.current_stream()
    cols = G * Z
    psi = torch.empty(D * cols, dtype=torch.float64, device="cuda")
    gdev.fill(psi, 0, gen.ARR_PSI, gdev.DIST_U01, LAYOUTS.index(lay), (D, G, Z))
    phi_in = torch.empty(NM * cols, dtype=torch.float64, device="cuda")
    gdev.fill(phi_in, 0, gen.ARR_PHI, gdev.DIST_SYM)
    phi = torch.empty(NM * cols, dtype=torch.float64, device="cuda")
    out = torch.empty(D * cols, dtype=torch.float64, device="cuda")
    L = gen.matrix_sym(0, gen.ARR_L, NM, D)
    Lp = gen.matrix_sym(0, gen.ARR_LPLUS, D, NM)
    half_L, half_Lp = L.copy(), Lp.copy()
    half_L[:, 1::2] = 0.0
    half_Lp[1::2, :] = 0.0
    pick = (np.arange(NM) * D) // NM
    oh_L = np.zeros((NM, D))
    oh_L[np.arange(NM), pick] = 1.0
    cases = {"dense": (L, Lp), "half_directions": (half_L, half_Lp), "onehot": (oh_L, oh_L.T.copy())}
    full = algorithmic_bytes(Z, G, D, NM)
    res = {}
    for name, (Lw, Lpw) in cases.items():
        L_d, Lp_d = torch.from_numpy(Lw.ravel().copy()).cuda(), torch.from_numpy(Lpw.ravel().copy()).cuda()
        for kern, W, W_d, x, y, kname in ((P.SJ_LTIMES, Lw, L_d, psi, phi, "ltimes"),
                                          (P.SJ_LPLUSTIMES, Lpw, Lp_d, phi_in, out, "lplustimes")):
            spec = dict(layout=lay, Z=Z, G=G, D=D, NM=NM)
            hv = P.sj_specialize_values(kern, W, **spec)
            hp = P.sj_specialize(kern, variant=P.SJ_VAR_DIRECT, order=1, **spec)
            hd = P.sj_specialize(kern, **spec)
            tv, _ = time_launches(lambda: P.sj_run(hv, [W_d, x, y]), a.steps, stream)
            yv = y.clone()
            tp, _ = time_launches(lambda: P.sj_run(hp, [W_d, x, y]), a.steps, stream)
            same = bool(torch.equal(yv, y))
            td, _ = time_launches(lambda: P.sj_run(hd, [W_d, x, y]), a.steps, stream)
            # rows of the streamed input some nonzero coefficient reaches
            needed_rows = int(np.count_nonzero(np.any(W != 0.0, axis=0)))   # columns of W = input rows
            in_rows = D if kern == P.SJ_LTIMES else NM
            out_rows = NM if kern == P.SJ_LTIMES else D
            need = (needed_rows + out_rows) * cols * 8 + NM * D * 8
            info = P.sj_handle_info(hv)
            res[f"{kname}_{name}"] = dict(
                values_us=round(tv * 1e3, 1), runtime_weights_us=round(tp * 1e3, 1), default_us=round(td * 1e3, 1),
                speedup_vs_runtime_weights=round(tp / tv, 3), speedup_vs_default=round(td / tv, 3),
                gbs_full_problem=round(full / (tv * 1e-3) / 1e9, 1), rows_read=needed_rows, rows_total=in_rows,
                gbs_rows_read=round(need / (tv * 1e-3) / 1e9, 1), bitwise_equal_to_runtime_weights=same,
                kernel=info["kernel_name"], compile_ms=round(info["compile_ms"], 1), code_bytes=info["code_bytes"],
                vgprs=info["vgprs"])
    dense = res["ltimes_dense"]
    line = {
        "metric": "LTimes/LPlusTimes with the weights compiled in (value specialization): GB/s and speedup over run-time weights",
        "value": dense["gbs_full_problem"], "unit": "GB/s", "n_gpus": 1, "steps": a.steps, "warmup": 0,
        "ms_per_step": round(dense["values_us"] / 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (SplitMix64, seed 0)",
        "config": {"workload": f"LTimes and LPlusTimes, DGZ, FP64, Z={Z} G={G} D={D} NM={NM}, weights as constants",
                   "weights": list(cases)},
        "roofline": {"bound": "hbm", "achieved": dense["gbs_full_problem"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dense["gbs_full_problem"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": dense["kernel"], "avg_us": dense["values_us"], "bytes_per_launch": full},
        "cases": res,
    }
    print(json.dumps(line), flush=True)


def bench_small(a):
    """LTimes and LPlusTimes, DGZ, FP64, Z=4096 G=8 D=48 NM=16: a launch moves
    16.8 MB, about 2 us at the HBM peak, so the launch and the cache lookup
    matter.  64 buffer sets (psi, phi, psi' each; 1.9 GB in all, so the launches
    cannot be served from the 256 MB last-level cache) are cycled through by 64
    launches captured in one HIP graph per operator; time per launch = graph
    replay time / 64.  Also the same 64 launches issued one by one, each after a
    cache lookup (sj_specialize hit), as a caller without graphs would."""
    import torch

    import paper_1904_08555_amd as P
    import sj_inputs as gen
    from sj_inputs import device as gdev

    Z, G, D, NM, nset = 4096, 8, 48, 16, 64
    stream = torch.cuda.current_stream()
    L_d = torch.empty(NM * D, dtype=torch.float64, device="cuda")
    Lp_d = torch.empty(D * NM, dtype=torch.float64, device="cuda")
    gdev.fill(L_d, 0, gen.ARR_L, gdev.DIST_SYM)
    gdev.fill(Lp_d, 0, gen.ARR_LPLUS, gdev.DIST_SYM)
    sets = []
    for _ in range(nset):
        psi = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
        gdev.fill(psi, 0, gen.ARR_PSI, gdev.DIST_U01, 0, (D, G, Z))
        sets.append((psi, torch.empty(NM * G * Z, dtype=torch.float64, device="cuda"),
                     torch.empty(D * G * Z, dtype=torch.float64, device="cuda")))
    # the specializations come from the exhaustive tuner, timed on this shape with a 1 GiB read
    # between launches (the launch's operands, 17 MB, would otherwise sit in the caches)
    tuned = {}
    if not a.no_tune:
        from paper_1904_08555_amd import tune
        flush = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
        for kname, kid, ptrs in (("ltimes", P.SJ_LTIMES, [L_d, sets[0][0], sets[0][1]]),
                                 ("lplustimes", P.SJ_LPLUSTIMES, [Lp_d, sets[0][1], sets[0][2]])):
            r = tune.tune_exhaustive(kid, "DGZ", Z, G, D, NM, ptrs, reps=10, warmup=2, flush=flush, threads=8)
            tuned[kname] = r["best"]
        del flush
    spec_l = P.make_spec(layout="DGZ", Z=Z, G=G, D=D, NM=NM, **tuned.get("ltimes", {}))
    spec_p = P.make_spec(layout="DGZ", Z=Z, G=G, D=D, NM=NM, **tuned.get("lplustimes", {}))
    h_l = P.sj_specialize(P.SJ_LTIMES, spec_l)
    h_p = P.sj_specialize(P.SJ_LPLUSTIMES, spec_p)
    nbytes = algorithmic_bytes(Z, G, D, NM)
    res = {}
    for name, h, kid, spec, ptrs in (
            ("ltimes", h_l, P.SJ_LTIMES, spec_l, [[L_d, s[0], s[1]] for s in sets]),
            ("lplustimes", h_p, P.SJ_LPLUSTIMES, spec_p, [[Lp_d, s[1], s[2]] for s in sets]),
            ("ltimes_default", P.sj_specialize(P.SJ_LTIMES, layout="DGZ", Z=Z, G=G, D=D, NM=NM), P.SJ_LTIMES,
             P.make_spec(layout="DGZ", Z=Z, G=G, D=D, NM=NM), [[L_d, s[0], s[1]] for s in sets]),
            ("lplustimes_default", P.sj_specialize(P.SJ_LPLUSTIMES, layout="DGZ", Z=Z, G=G, D=D, NM=NM),
             P.SJ_LPLUSTIMES, P.make_spec(layout="DGZ", Z=Z, G=G, D=D, NM=NM), [[Lp_d, s[1], s[2]] for s in sets])):
        for p in ptrs:                                   # warm up, outside capture
            P.sj_run(h, p)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for p in ptrs:
                P.sj_run(h, p)
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        per = []
        for _ in range(max(5, a.steps)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g.replay()
            e1.record(stream)
            per.append((e0, e1))
        torch.cuda.synchronize()
        g_ms = statistics.median(x.elapsed_time(y) for x, y in per) / nset
        # one by one, each launch after a lookup (hit) of its specialization, no graph
        lib = P.lib()
        hout = ctypes.c_void_p()
        arrs = [(ctypes.c_void_p * 3)(*(t.data_ptr() for t in p)) for p in ptrs]
        sref = ctypes.byref(spec)
        sptr = stream.cuda_stream
        walls = []
        for _ in range(max(5, a.steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for arr in arrs:
                lib.sj_specialize(kid, sref, ctypes.byref(hout))
                lib.sj_run(hout, arr, 3, sptr)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        e_ms = statistics.median(walls) * 1e3 / nset
        res[name] = dict(graph_us_per_launch=round(g_ms * 1e3, 3),
                         graph_gbs=round(nbytes / (g_ms * 1e-3) / 1e9, 1),
                         graph_frac=round(nbytes / (g_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         eager_with_lookup_us_per_launch=round(e_ms * 1e3, 3),
                         kernel=P.sj_handle_info(h)["kernel_name"], src_sha1=source_sha1(P, kid, spec),
                         traffic=measured_traffic(P, kid, spec))
        del g
    # the floor: the same graph of 64 dependent launches of a one-column LTimes (one workgroup, 8 bytes
    # of psi), i.e. what a launch costs in this graph with no data to move
    tiny = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(3)]
    h_t = P.sj_specialize(P.SJ_LTIMES, layout="DGZ", Z=1, G=1, D=1, NM=1)
    P.sj_run(h_t, tiny)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(nset):
            P.sj_run(h_t, tiny)
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    per = []
    for _ in range(max(5, a.steps)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.replay()
        e1.record(stream)
        per.append((e0, e1))
    torch.cuda.synchronize()
    floor_us = statistics.median(x.elapsed_time(y) for x, y in per) / nset * 1e3
    del g
    tot = res["ltimes"]["graph_us_per_launch"] + res["lplustimes"]["graph_us_per_launch"]
    line = {
        "metric": "LTimes + LPlusTimes per-launch time at the small DGZ shape (HIP graph of 64 launches)",
        "value": round(2 * nbytes / (tot * 1e-6) / 1e9, 1), "unit": "GB/s", "n_gpus": 1, "steps": a.steps,
        "warmup": 3, "ms_per_step": round(tot * 1e-3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (SplitMix64 counter generator, seed 0)",
        "config": {"workload": f"LTimes+LPlusTimes, DGZ, FP64, Z={Z} G={G} D={D} NM={NM}",
                   "buffer_sets": nset, "launches_per_graph": nset,
                   "specialization": "exhaustive tuner" if tuned else "library defaults"},
        "tuned": tuned,
        "roofline": {"bound": "hbm", "achieved": res["ltimes"]["graph_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": res["ltimes"]["graph_frac"], "traffic": res["ltimes"]["traffic"], "kernel": res["ltimes"]["kernel"],
                     "avg_us": res["ltimes"]["graph_us_per_launch"], "bytes_per_launch": nbytes},
        "per_kernel": res,
        "launch_floor_us": round(floor_us, 3),
        "floor_note": ("per-launch time of the same graph with a one-column LTimes: what a dependent launch "
                       "costs here with no data to move"),
    }
    print(json.dumps(line), flush=True)


def bench_scattering(a):
    """Scattering source phi_out[nm,g,z] = sum_g' S[mat(z)][n(nm)][g][g'] phi[nm,g',z]
    over the six nestings, FP64, Z=32768 G=32 NM=16 (degrees 0..3), four
    materials in contiguous zone regions; also every zone's material drawn at
    random (per-lane matrices) for one nesting.  value = algorithmic bytes of
    the six launches / their summed median times."""
    import math

    import numpy as np
    import torch

    import paper_1904_08555_amd as P
    import sj_inputs as gen
    from sj_inputs import device as gdev

    Z, G, NM, nmat = a.Z, a.G, a.NM, 4
    layouts = [x for x in a.layouts.split(",") if x] or list(LAYOUTS)
    stream = torch.cuda.current_stream()
    nl = math.isqrt(NM - 1) + 1
    rng = np.random.default_rng(0)
    S_d = torch.from_numpy(rng.uniform(0.0, 1.0 / G, (nmat, nl, G, G)).ravel()).cuda()
    mat_reg = torch.from_numpy(((np.arange(Z) * nmat) // Z).astype(np.int32)).cuda()
    mat_rnd = torch.from_numpy(rng.integers(0, nmat, Z).astype(np.int32)).cuda()
    phi = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
    out = torch.empty_like(phi)
    # phi and phi_out together (268 MB) are about the size of the 256 MB last-level cache: a 1 GiB
    # scratch buffer is read before every timed launch (outside its events)
    flush = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
    nbytes = 2 * NM * G * Z * 8 + S_d.numel() * 8 + Z * 4
    res, tot = {}, 0.0
    for lay in layouts:
        gdev.fill(phi, 0, gen.ARR_PHI, gdev.DIST_U01, LAYOUTS.index(lay), (NM, G, Z))
        spec = P.make_spec(layout=lay, Z=Z, G=G, NM=NM, count=nmat)
        h = P.sj_specialize(P.SJ_SCATTERING, spec)
        t, _ = time_launches(lambda: P.sj_run(h, [S_d, mat_reg, phi, out]), a.steps, stream, flush, warmup=40)
        tr, _ = time_launches(lambda: P.sj_run(h, [S_d, mat_rnd, phi, out]), max(3, a.steps // 4), stream, flush)
        info = P.sj_handle_info(h)
        tot += t
        res[lay] = dict(us=round(t * 1e3, 1), gbs=round(nbytes / (t * 1e-3) / 1e9, 1),
                        frac=round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        random_materials_us=round(tr * 1e3, 1), kernel=info["kernel_name"], vgprs=info["vgprs"],
                        tile_n=info["tile_n"], block=info["block"], order=info.get("order"),
                        compile_ms=round(info["compile_ms"], 1), src_sha1=source_sha1(P, P.SJ_SCATTERING, spec),
                        traffic=measured_traffic(P, P.SJ_SCATTERING, spec))
        if info["variant"] == P.SJ_VAR_DIRECT:   # the matrix-core structure of this nesting beside it, if any
            try:
                hm = P.sj_specialize(P.SJ_SCATTERING, P.make_spec(layout=lay, Z=Z, G=G, NM=NM, count=nmat,
                                                                  variant=P.SJ_VAR_MFMA))
            except P.SJError:
                hm = None
            if hm is not None:
                tm, _ = time_launches(lambda: P.sj_run(hm, [S_d, mat_reg, phi, out]), a.steps, stream, flush,
                                      warmup=10)
                tmr, _ = time_launches(lambda: P.sj_run(hm, [S_d, mat_rnd, phi, out]), max(3, a.steps // 4), stream,
                                       flush)
                res[lay].update(mfma_us=round(tm * 1e3, 1), mfma_random_materials_us=round(tmr * 1e3, 1),
                                mfma_kernel=P.sj_handle_info(hm)["kernel_name"])
        if info["variant"] != P.SJ_VAR_DIRECT:   # the vector-FMA structure of this nesting beside it
            hd = P.sj_specialize(P.SJ_SCATTERING, P.make_spec(layout=lay, Z=Z, G=G, NM=NM, count=nmat,
                                                              variant=P.SJ_VAR_DIRECT))
            td, _ = time_launches(lambda: P.sj_run(hd, [S_d, mat_reg, phi, out]), a.steps, stream, flush, warmup=10)
            tdr, _ = time_launches(lambda: P.sj_run(hd, [S_d, mat_rnd, phi, out]), max(3, a.steps // 4), stream,
                                   flush)
            res[lay].update(direct_us=round(td * 1e3, 1), direct_random_materials_us=round(tdr * 1e3, 1),
                            direct_kernel=P.sj_handle_info(hd)["kernel_name"],
                            speedup_vs_direct=round(td / t, 3))
    dom = max(res, key=lambda k: res[k]["us"])
    # the device-copy rate at this size (phi to phi_out, the same scratch read before each copy): the
    # practical ceiling of a launch that reads and writes 134 MB each
    cmed, _ = time_launches(lambda: out.copy_(phi), max(5, a.steps // 2), stream, flush, warmup=2)
    copy_gbs = 2 * phi.numel() * 8 / (cmed * 1e-3) / 1e9
    line = {
        "metric": "scattering source GB/s over six nestings (specialized kernels)",
        "value": round(nbytes * len(layouts) / (tot * 1e-3) / 1e9, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": a.steps, "warmup": 0, "ms_per_step": round(tot, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (SplitMix64 phi, seeded S and materials)",
        "config": {"workload": f"scattering, FP64, Z={Z} G={G} NM={NM}, {nmat} materials in zone regions",
                   "layouts": layouts, "cache": "1 GiB scratch read before every timed launch"},
        "roofline": {"bound": "hbm", "achieved": res[dom]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": res[dom]["frac"], "traffic": res[dom]["traffic"], "kernel": res[dom]["kernel"],
                     "avg_us": res[dom]["us"], "bytes_per_launch": nbytes, "measured_copy_gbs": round(copy_gbs, 1),
                     "frac_of_measured_copy": round(res[dom]["gbs"] / copy_gbs, 4)},
        "per_layout": res,
    }
    print(json.dumps(line), flush=True)


def bench_mass(a):
    """Tensor-product mass operator (partial assembly): hexahedra with D1D = 4
    dofs and Q1D = 6 points per direction (500,000 elements) and quadrilaterals
    with D1D = 4, Q1D = 6 (2,000,000 elements), FP64.  The specialization fixes
    dim, D1D, Q1D and the element count.  value = algorithmic bytes (x and the
    point data read, y written, B1 once) of both launches / their median times."""
    import numpy as np
    import torch

    import paper_1904_08555_amd as P

    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(0)
    res, tot_b, tot_t = {}, 0, 0.0
    for dim, D1D, Q1D, NE in ((3, 4, 6, 500000), (2, 4, 6, 2000000)):
        nd, nq = D1D ** dim, Q1D ** dim
        B1 = torch.from_numpy(rng.uniform(-1, 1, Q1D * D1D)).cuda()
        g = torch.Generator("cuda").manual_seed(0)
        Dq = torch.rand(NE * nq, dtype=torch.float64, device="cuda", generator=g)
        X = torch.rand(NE * nd, dtype=torch.float64, device="cuda", generator=g)
        Y = torch.empty_like(X)
        spec = P.make_spec(D=D1D, NM=Q1D, inputs=dim, count=NE)
        h = P.sj_specialize(P.SJ_MASS, spec)
        # 40 untimed launches first: the first few dozen run up to 25% slower (measured 338 us, then
        # 274 us for the same hexahedral kernel)
        t, _ = time_launches(lambda: P.sj_run(h, [B1, Dq, X, Y]), a.steps, stream, warmup=40)
        nb = NE * (2 * nd + nq) * 8 + Q1D * D1D * 8
        flops = 2 * NE * 2 * sum(D1D ** (dim - s) * Q1D ** (s + 1) for s in range(dim)) if dim > 0 else 0
        info = P.sj_handle_info(h)
        res[f"{dim}d_d{D1D}_q{Q1D}_ne{NE}"] = dict(us=round(t * 1e3, 1), gbs=round(nb / (t * 1e-3) / 1e9, 1),
                                                   frac=round(nb / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                                   gflops=round(flops / (t * 1e-3) / 1e9, 1), bytes=nb,
                                                   kernel=info["kernel_name"], elements_per_wave=info["tile_n"],
                                                   block=info["block"], vgprs=info["vgprs"], lds=info["lds_bytes"],
                                                   src_sha1=source_sha1(P, P.SJ_MASS, spec),
                                                   traffic=measured_traffic(P, P.SJ_MASS, spec))
        tot_b += nb
        tot_t += t
        del Dq, X, Y
    dom = max(res, key=lambda k: res[k]["us"])
    line = {
        "metric": "tensor-product mass operator (partial assembly) GB/s",
        "value": round(tot_b / (tot_t * 1e-3) / 1e9, 1), "unit": "GB/s", "n_gpus": 1, "steps": a.steps,
        "warmup": 0, "ms_per_step": round(tot_t, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (torch Philox U[0,1) x and point data, seeded B1)",
        "config": {"workload": "mass operator y_e = B^T D_e B x_e: hex D1D=4 Q1D=6 NE=500000; quad D1D=4 Q1D=6 NE=2000000"},
        "roofline": {"bound": "hbm", "achieved": res[dom]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": res[dom]["frac"], "traffic": res[dom]["traffic"], "kernel": res[dom]["kernel"], "avg_us": res[dom]["us"],
                     "bytes_per_launch": res[dom]["bytes"]},
        "cases": res,
    }
    print(json.dumps(line), flush=True)


def bench_fused(a):
    """LTimes then LPlusTimes per nesting as one fused pass (phi kept in
    registers; written out too, or not) against the two separate kernels, FP64,
    Z=32768 G=32 D=96 NM=16, default specializations.  value = algorithmic
    bytes of the fused step (with phi written) / its time."""
    import torch

    import paper_1904_08555_amd as P
    import sj_inputs as gen
    from sj_inputs import device as gdev

    Z, G, D, NM = a.Z, a.G, a.D, a.NM
    layouts = [x for x in a.layouts.split(",") if x] or list(LAYOUTS)
    stream = torch.cuda.current_stream()
    L_d = torch.empty(NM * D, dtype=torch.float64, device="cuda")
    Lp_d = torch.empty(D * NM, dtype=torch.float64, device="cuda")
    gdev.fill(L_d, 0, gen.ARR_L, gdev.DIST_SYM)
    gdev.fill(Lp_d, 0, gen.ARR_LPLUS, gdev.DIST_SYM)
    psi = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
    phi = torch.empty(NM * G * Z, dtype=torch.float64, device="cuda")
    out = torch.empty(D * G * Z, dtype=torch.float64, device="cuda")
    cols = G * Z
    b_with = (2 * D + NM) * cols * 8 + 2 * NM * D * 8
    b_without = 2 * D * cols * 8 + 2 * NM * D * 8
    b_sep = 2 * algorithmic_bytes(Z, G, D, NM)
    res = {}
    tot_fused, tot_sep = 0.0, 0.0
    for lay in layouts:
        gdev.fill(psi, 0, gen.ARR_PSI, gdev.DIST_U01, LAYOUTS.index(lay), (D, G, Z))
        fspec = P.make_spec(layout=lay, Z=Z, G=G, D=D, NM=NM)
        hf = P.sj_specialize(P.SJ_LTIMES_LPLUS, fspec)
        h1 = P.sj_specialize(P.SJ_LTIMES, layout=lay, Z=Z, G=G, D=D, NM=NM)
        h2 = P.sj_specialize(P.SJ_LPLUSTIMES, layout=lay, Z=Z, G=G, D=D, NM=NM)

        def sep():
            P.sj_run(h1, [L_d, psi, phi])
            P.sj_run(h2, [Lp_d, phi, out])
        fused_with, _ = time_launches(lambda: P.sj_run(hf, [L_d, Lp_d, psi, out, phi]), a.steps, stream)
        fused_without, _ = time_launches(lambda: P.sj_run(hf, [L_d, Lp_d, psi, out]), a.steps, stream)
        sep_ms, _ = time_launches(sep, a.steps, stream)
        tot_fused += fused_with
        tot_sep += sep_ms
        res[lay] = dict(fused_us=round(fused_with * 1e3, 1), fused_gbs=round(b_with / (fused_with * 1e-3) / 1e9, 1),
                        fused_no_phi_us=round(fused_without * 1e3, 1),
                        fused_no_phi_gbs=round(b_without / (fused_without * 1e-3) / 1e9, 1),
                        separate_us=round(sep_ms * 1e3, 1), speedup=round(sep_ms / fused_with, 3),
                        kernel=P.sj_handle_info(hf)["kernel_name"],
                        src_sha1=source_sha1(P, P.SJ_LTIMES_LPLUS, fspec),
                        traffic=measured_traffic(P, P.SJ_LTIMES_LPLUS, fspec))
    dom = max(res, key=lambda k: res[k]["fused_us"])
    line = {
        "metric": "fused LTimes+LPlusTimes GB/s (phi kept on chip) vs the two separate kernels",
        "value": round(b_with * len(layouts) / (tot_fused * 1e-3) / 1e9, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": a.steps, "warmup": 0, "ms_per_step": round(tot_fused, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (SplitMix64, seed 0)",
        "config": {"workload": f"psi -> phi -> psi' per nesting, FP64, Z={Z} G={G} D={D} NM={NM}", "layouts": layouts},
        "roofline": {"bound": "hbm", "achieved": res[dom]["fused_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(res[dom]["fused_gbs"] / HBM_PEAK_GBS, 4), "traffic": res[dom]["traffic"],
                     "kernel": res[dom]["kernel"], "avg_us": res[dom]["fused_us"], "bytes_per_launch": b_with},
        "separate_ms_per_step": round(tot_sep, 4), "speedup_vs_separate": round(tot_sep / tot_fused, 3),
        "bytes": {"fused_with_phi": b_with, "fused_without_phi": b_without, "separate_pair": b_sep},
        "per_layout": res,
    }
    print(json.dumps(line), flush=True)


def bench_copy(a):
    """Plain device-to-device copy of 1 GiB (known traffic: 1 GiB read and
    1 GiB written per dispatch).  Used to calibrate the FETCH_SIZE and
    WRITE_SIZE counters against which the kernels' HBM traffic is scaled."""
    import torch
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    med, mean = time_launches(lambda: dst.copy_(src), max(3, a.steps), stream)
    line = {"metric": "device copy GB/s (read + write)", "value": round(2 * n * 8 / (med * 1e-3) / 1e9, 1),
            "unit": "GB/s", "n_gpus": 1, "steps": a.steps, "warmup": 0, "ms_per_step": round(med, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "ones",
            "config": {"workload": "copy 1 GiB float64", "read_bytes": n * 8, "write_bytes": n * 8}}
    print(json.dumps(line), flush=True)


def bench_picker(a):
    """Learned picker against the exhaustive tuner: 250 training shapes x 8
    random candidates = 2000 timed training configurations (and, beside it,
    the same evaluation with 500 more training shapes: 6000); 200 held-out
    shapes, each timed over the tuner's whole candidate set C(s) (every
    nesting's tune.candidates); regret of the pick and of the spread-based
    shortlist against the tuner's best, compiles needed, and speedup over the
    untuned default.  --picker-part collect gathers timings into
    out-dir/picker_data_<lo>_<hi>.json for --picker-slice lo:hi (held-out
    shapes lo..hi-1) or out-dir/picker_data_train.json for --picker-slice train,
    so that the collection can be split over several runs; --picker-part
    evaluate trains and scores on the files named by --picker-data."""
    from paper_1904_08555_amd import picker

    t0 = time.perf_counter()
    os.makedirs(a.out_dir, exist_ok=True)
    log = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
    if a.picker_part == "collect" and a.picker_slice == "train":
        lo, hi, train, name = 0, 0, "only", "train"
    else:
        lo, hi = (int(x) for x in a.picker_slice.split(":")) if a.picker_slice else (0, 200)
        train, name = a.picker_part == "all", f"{lo}_{hi}"
    if a.picker_part in ("all", "collect"):
        data = picker.collect(n_train_shapes=250, per_shape=8, n_eval=200, seed=0, workers=12, log=log,
                              eval_slice=(lo, hi), train=train, extra_train_shapes=500)
        path = os.path.join(a.out_dir, f"picker_data_{name}.json")
        with open(path, "w") as f:
            json.dump(data, f)
        if a.picker_part == "collect":
            print(json.dumps({"picker_collect": path, "train": len(data.get("train", [])),
                              "eval_shapes": len(data["eval"]), "train_collect_s": data.get("train_collect_s"),
                              "eval_collect_s": data.get("eval_collect_s"),
                              "wall_s": round(time.perf_counter() - t0, 1)}), flush=True)
            return
        parts = [data]
    else:
        parts = []
        for path in a.picker_data.split(","):
            with open(path) as f:
                parts.append(json.load(f))
    data = dict(train=[], eval=[])
    for d in parts:
        data["train"] += d.get("train", [])
        data["eval"] += d["eval"]
    # the headline: 2000 timed training configurations (the 250 shapes drawn before the held-out
    # ones, 8 candidates each); then the same held-out evaluation with all 6000
    base = {json.dumps(s, sort_keys=True) for s in picker.experiment_shapes(250, 200, seed=0)[0]}
    data_base = dict(train=[x for x in data["train"] if json.dumps(x[0], sort_keys=True) in base], eval=data["eval"])
    res, _, rows = picker.evaluate(data_base, seed=0, epochs=200, log=log)
    res_all, pk_all, rows_all = picker.evaluate(data, seed=0, epochs=200, log=log)
    for r in (res, res_all):
        r["train_collect_s"] = sum(d.get("train_collect_s") or 0 for d in parts)
        r["eval_collect_s"] = sum(d.get("eval_collect_s") or 0 for d in parts)
    wall = time.perf_counter() - t0
    pk_all.save(os.path.join(a.out_dir, "picker_weights.json"))
    pk_all.save(os.path.join(a.out_dir, "picker_weights.npz"))   # the form shipped as picker.PRETRAINED
    with open(os.path.join(a.out_dir, "picker_rows.json"), "w") as f:
        json.dump(rows, f)
    with open(os.path.join(a.out_dir, "picker_rows_6000.json"), "w") as f:
        json.dump(rows_all, f)
    line = {
        "metric": "picker regret vs exhaustive autotuner (mean over held-out shapes)",
        "value": res["regret_mean"], "unit": "fraction", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(wall * 1e3, 1), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 model; f64 and bf16x3 kernels", "data": "synthetic (SplitMix64 + timings gathered here)",
        "config": {"workload": "picker: 2000 timed training configs (250 shapes x 8 candidates), 200 held-out "
                               "shapes each timed over the exhaustive tuner's candidate set; Z=k^3 k in 8..64, "
                               "G in 8..128, D in 16..256 step 8, NM in {4,9,16,36,64}, dtype in {f64, bf16x3}"},
        "roofline": None, "cpu_baseline": None, "picker": res,
        "picker_6000_training_configs": res_all,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
