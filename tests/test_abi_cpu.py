"""CPU tests of the C ABI: the library loads and exports every entry point the
header declares; keys canonicalize; the cache compiles each key once, also
under concurrency; errors come back as status codes with messages.  Compiles
here use SJ_FLAG_COMPILE_ONLY (hiprtc needs no GPU when the target is given);
nothing is launched."""
import os
import re
import threading

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_1904_08555_amd as P
    P.lib()
    return P


def header_entry_points():
    with open(os.path.join(ROOT, "include", "sj.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^(?:sj_status|const char \*)\s*(sj_[a-z0-9_]+)\(", text, re.M)))


def test_exports_every_declared_symbol(P):
    names = header_entry_points()
    assert len(names) >= 18
    lib = P.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(P.EXPORTED)


def test_struct_sizes_match_header(P):
    """The ctypes mirrors must have the C sizes (checked through struct_size validation)."""
    import ctypes
    s = P.make_spec(layout="DGZ", Z=4, G=2, D=3, NM=2, flags=P.SJ_FLAG_COMPILE_ONLY)
    src = P.sj_emit_source(P.SJ_LTIMES, s)
    assert "SJ_D 3" in src
    s.struct_size = ctypes.sizeof(P.sj_spec) + 8
    with pytest.raises(P.SJError) as e:
        P.sj_emit_source(P.SJ_LTIMES, s)
    assert e.value.status == P.SJ_ERR_INVALID_ARG


def test_layout_strings(P):
    for i, name in enumerate(P.LAYOUTS):
        assert P.sj_layout_from_string(name) == i
        assert P.sj_layout_from_string(name.lower()) == i
    for bad in ("", "DG", "DGZZ", "XYZ", "DDD"):
        with pytest.raises(P.SJError) as e:
            P.sj_layout_from_string(bad)
        assert e.value.status == P.SJ_ERR_INVALID_ARG


def test_emitted_source_is_self_contained(P):
    for layout in P.LAYOUTS:
        for k in (P.SJ_LTIMES, P.SJ_LPLUSTIMES):
            src = P.sj_emit_source(k, layout=layout, Z=32768, G=32, D=96, NM=16)
            assert "#include" not in src
            assert "SJ_D 96" in src and "SJ_NM 16" in src
    big = P.sj_emit_source(P.SJ_LTIMES, layout="DGZ", Z=262144, G=64, D=128, NM=16)
    assert "typedef long long sj_index_t" in big        # 2^31 elements -> 64-bit indexing
    small = P.sj_emit_source(P.SJ_LTIMES, layout="DGZ", Z=4096, G=8, D=48, NM=16)
    assert "typedef int sj_index_t" in small


@pytest.mark.parametrize("bad", [
    dict(Z=0), dict(G=-1), dict(D=2 ** 31), dict(NM=0), dict(layout=6), dict(dtype=9),
    dict(block=100), dict(block=2048), dict(tile_n=3, variant=1, layout="DGZ"), dict(tile_n=9),
    dict(unroll=0, variant=1, tile_n=5), dict(order=3, variant=1, layout="DGZ"), dict(order=2, D=9), dict(order=2, variant=2),
    dict(variant=2, layout="DGZ"), dict(variant=9),
])
def test_invalid_specs_rejected(P, bad):
    spec = dict(layout="ZGD", Z=10, G=3, D=8, NM=4, flags=P.SJ_FLAG_COMPILE_ONLY)
    spec.update(bad)
    with pytest.raises(P.SJError) as e:
        P.sj_specialize(P.SJ_LTIMES, **spec)
    assert e.value.status in (P.SJ_ERR_INVALID_ARG, P.SJ_ERR_UNSUPPORTED)
    assert P.sj_last_error()


def test_compile_only_cache_and_canonical_keys(P):
    s0 = P.sj_stats()
    h1 = P.sj_specialize(P.SJ_LTIMES, layout="DZG", Z=40, G=6, D=9, NM=5, flags=P.SJ_FLAG_COMPILE_ONLY)
    # explicit defaults and a lower-case layout name canonicalize to the same key
    h2 = P.sj_specialize(P.SJ_LTIMES, layout="dzg", Z=40, G=6, D=9, NM=5, block=256, tile_n=2, unroll=8,
                         flags=P.SJ_FLAG_COMPILE_ONLY)
    assert h1 == h2
    s1 = P.sj_stats()
    assert s1["compiles"] - s0["compiles"] == 1
    assert s1["hits"] - s0["hits"] == 1
    info = P.sj_handle_info(h1)
    assert info["kernel_name"] == "sj_ltimes_direct_dzg"
    assert info["compile_ms"] > 0 and info["code_bytes"] > 1000
    assert info["vgprs"] > 0 and info["sgprs"] > 0 and info["scratch_bytes"] == 0
    code = P.sj_handle_code(h1)
    assert code[:4] == b"\x7fELF"
    # a compile-only handle cannot run
    with pytest.raises(P.SJError) as e:
        P.sj_run(h1, [16, 32, 48])
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    # a different tile is a different key
    h3 = P.sj_specialize(P.SJ_LTIMES, layout="DZG", Z=40, G=6, D=9, NM=5, unroll=3, flags=P.SJ_FLAG_COMPILE_ONLY)
    assert h3 != h1


def test_concurrent_requests_compile_once(P):
    s0 = P.sj_stats()
    spec = dict(layout="GDZ", Z=77, G=5, D=11, NM=3, flags=P.SJ_FLAG_COMPILE_ONLY)
    out = []
    errs = []

    def worker():
        try:
            out.append(P.sj_specialize(P.SJ_LPLUSTIMES, **spec))
        except Exception as e:  # pragma: no cover - reported below
            errs.append(e)

    ts = [threading.Thread(target=worker) for _ in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errs
    assert len(set(out)) == 1
    s1 = P.sj_stats()
    assert s1["compiles"] - s0["compiles"] == 1
    assert (s1["hits"] - s0["hits"]) == 7
    assert s1["inflight_waits"] - s0["inflight_waits"] >= 1


def test_forced_compile_error_leaves_no_entry(P):
    spec = dict(layout="DGZ", Z=9, G=2, D=4, NM=2, flags=P.SJ_FLAG_COMPILE_ONLY | P.SJ_FLAG_DEBUG_FAIL_COMPILE)
    s0 = P.sj_stats()
    for _ in range(2):
        with pytest.raises(P.SJError) as e:
            P.sj_specialize(P.SJ_LTIMES, **spec)
        assert e.value.status == P.SJ_ERR_COMPILE
        assert "SJ_FLAG_DEBUG_FAIL_COMPILE" in e.value.message   # the compiler log is returned
    s1 = P.sj_stats()
    assert s1["compile_failures"] - s0["compile_failures"] == 2   # retried, not cached
    assert s1["entries"] == s0["entries"]


def test_generic_run_validates_before_launch(P):
    with pytest.raises(P.SJError) as e:
        P.sj_generic_run(P.SJ_LTIMES, [16, 32, 48], layout="DGZ", Z=0, G=1, D=1, NM=1)
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    with pytest.raises(P.SJError) as e:
        P.sj_generic_run(P.SJ_LTIMES, [16, 32, 48], layout="DGZ", Z=1, G=1, D=1, NM=1, dtype=P.SJ_BF16)
    assert e.value.status == P.SJ_ERR_UNSUPPORTED
    with pytest.raises(P.SJError) as e:
        P.sj_generic_run(P.SJ_LTIMES, [16, 40, 48], layout="DGZ", Z=1, G=1, D=1, NM=1)
    assert e.value.status == P.SJ_ERR_ALIGN
    with pytest.raises(P.SJError) as e:   # output range overlaps the input range
        P.sj_generic_run(P.SJ_LTIMES, [16, 4096, 4096 + 16], layout="DGZ", Z=4, G=1, D=4, NM=4)
    assert e.value.status == P.SJ_ERR_ALIAS


def test_product_path_has_no_oracle_dependency():
    """The product package and its C sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1904_08555_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h", ".hipk")):
                with open(os.path.join(dirpath, fn)) as f:
                    text = f.read()
                assert "oracle" not in text.lower(), os.path.join(dirpath, fn)


def test_bgemm_and_mlp_specs_compile(P):
    h = P.sj_specialize(P.SJ_BGEMM, flags=P.SJ_FLAG_COMPILE_ONLY)
    info = P.sj_handle_info(h)
    assert info["kernel_name"] == "sj_bgemm_persistent" and info["scratch_bytes"] == 0
    src = P.sj_emit_source(P.SJ_BGEMM, class_mask=(1 << 3) | (1 << 9))
    assert "sj_bgemm_class<3>" in src and "sj_bgemm_class<9>" in src and "sj_bgemm_class<4>" not in src
    for k in (P.SJ_MLP_FWD, P.SJ_MLP_BWD):
        h = P.sj_specialize(k, dtype=P.SJ_F32, rows=64, inputs=24, width=64, flags=P.SJ_FLAG_COMPILE_ONLY)
        assert P.sj_handle_info(h)["scratch_bytes"] == 0
    h = P.sj_specialize(P.SJ_ADAM, dtype=P.SJ_F32, rows=1000, flags=P.SJ_FLAG_COMPILE_ONLY)
    assert P.sj_handle_info(h)["kernel_name"] == "sj_adam"


@pytest.mark.parametrize("kernel,bad", [
    ("SJ_BGEMM", dict(class_mask=1)), ("SJ_BGEMM", dict(unroll=3)), ("SJ_BGEMM", dict(dtype=1)),
    ("SJ_BGEMM", dict(tile_n=-1)), ("SJ_BGEMM", dict(tile_k=2)), ("SJ_BGEMM", dict(order=5)),
    ("SJ_MLP_FWD", dict(dtype=3, rows=0, inputs=4, width=4)), ("SJ_MLP_FWD", dict(dtype=3, rows=4, inputs=65, width=4)),
    ("SJ_MLP_BWD", dict(dtype=0, rows=4, inputs=4, width=4)), ("SJ_ADAM", dict(dtype=3, rows=0)),
])
def test_bgemm_mlp_invalid_specs(P, kernel, bad):
    spec = dict(flags=P.SJ_FLAG_COMPILE_ONLY)
    spec.update(bad)
    with pytest.raises(P.SJError) as e:
        P.sj_specialize(getattr(P, kernel), **spec)
    assert e.value.status in (P.SJ_ERR_INVALID_ARG, P.SJ_ERR_UNSUPPORTED)


def test_mlp_workspace_offsets_fit_32_bits(P):
    """The MLP kernels index their rows * (4 width + 2) workspace with 32-bit
    offsets: a shape that would wrap is refused before any compile; the largest
    accepted row count at width 64 still fits."""
    width = 64
    limit = (1 << 31) // (4 * width + 2)          # rows * 258 < 2^31  <=>  rows <= limit (2^31 is not a multiple)
    for k in (P.SJ_MLP_FWD, P.SJ_MLP_BWD):
        with pytest.raises(P.SJError) as e:
            P.sj_specialize(k, dtype=P.SJ_F32, rows=limit + 1, inputs=24, width=width, flags=P.SJ_FLAG_COMPILE_ONLY)
        assert e.value.status == P.SJ_ERR_INVALID_ARG and "2^31" in str(e.value)
    assert limit * (4 * width + 2) < (1 << 31) <= (limit + 1) * (4 * width + 2)
    src = P.sj_emit_source(P.SJ_MLP_BWD, dtype=P.SJ_F32, rows=limit, inputs=24, width=width)
    assert f"#define SJ_R {limit}" in src


def test_mass_accepted_range(P):
    """D1D and Q1D in [1, 32]; for dim 3 the per-wave LDS tiles of one element,
    (2 max(D1D, Q1D)^3 + Q1D^3) doubles, must fit 160 KiB: 18 fits, 19 does not."""
    for dim, n in ((1, 32), (2, 32), (3, 18)):
        P.sj_emit_source(P.SJ_MASS, D=n, NM=n, inputs=dim, count=3)
    with pytest.raises(P.SJError) as e:
        P.sj_emit_source(P.SJ_MASS, D=19, NM=19, inputs=3, count=3)
    assert e.value.status == P.SJ_ERR_UNSUPPORTED
    with pytest.raises(P.SJError) as e:
        P.sj_emit_source(P.SJ_MASS, D=33, NM=4, inputs=1, count=3)
    assert e.value.status == P.SJ_ERR_INVALID_ARG


def test_compile_farm_matches_local_compile(P):
    """Worker processes produce the same code object the parent compiles."""
    from paper_1904_08555_amd import farm
    spec = dict(layout="GDZ", Z=123, G=7, D=24, NM=9)
    with farm.CompileFarm(2) as f:
        res = f.compile([(P.SJ_LTIMES, spec), (P.SJ_LTIMES, dict(spec, Z=0))])
    code, ms, err = res[0]
    assert err is None and code[:4] == b"\x7fELF" and ms > 0
    assert res[1][0] is None and res[1][2][0] == P.SJ_ERR_INVALID_ARG
    local = P.sj_handle_code(P.sj_specialize(P.SJ_LTIMES, flags=P.SJ_FLAG_COMPILE_ONLY, **spec))
    # comgr embeds per-compile temporary names, so bytes differ; size and symbol agree
    assert len(local) == len(code) and b"sj_ltimes_direct" in code and b"sj_ltimes_direct" in local


def test_specialize_with_code_rejects_garbage(P):
    with pytest.raises(P.SJError) as e:
        P.sj_specialize_with_code(P.SJ_LTIMES, b"not a code object", layout="DGZ", Z=1, G=1, D=1, NM=1)
    assert e.value.status in (P.SJ_ERR_LOAD, P.SJ_ERR_NOT_INITIALIZED)


def test_matrix_core_column_and_bf16_specs(P):
    """FP64 MFMA column kernel and BF16 forms: names, resolved tiles and
    rejected tiles, compiled without a GPU."""
    base = dict(Z=4096, G=8, D=48, NM=16, flags=P.SJ_FLAG_COMPILE_ONLY)
    h = P.sj_specialize(P.SJ_LTIMES, layout="GDZ", variant=P.SJ_VAR_MFMA, **base)
    info = P.sj_handle_info(h)
    assert info["kernel_name"] == "sj_ltimes_cols_mfma_gdz" and info["tile_n"] == 4 and info["scratch_bytes"] == 0
    h = P.sj_specialize(P.SJ_LPLUSTIMES, layout="ZDG", variant=P.SJ_VAR_MFMA, **base)
    info = P.sj_handle_info(h)
    # 48 outputs per column = 3 blocks of 16: the accumulator budget allows 2 columns per lane
    assert info["kernel_name"] == "sj_lplustimes_cols_mfma_zdg" and info["tile_n"] == 2
    src = P.sj_emit_source(P.SJ_LTIMES, layout="DGZ", variant=P.SJ_VAR_MFMA, order=2, unroll=3, **base)
    assert "#define SJ_ROTATE 1" in src and "#define SJ_PF 3" in src
    for bad in (dict(tile_n=3), dict(unroll=17), dict(order=5)):
        with pytest.raises(P.SJError) as e:
            P.sj_specialize(P.SJ_LTIMES, layout="DGZ", variant=P.SJ_VAR_MFMA, **dict(base, **bad))
        assert e.value.status == P.SJ_ERR_INVALID_ARG
    with pytest.raises(P.SJError) as e:   # 4 columns per lane need the contiguous extent % 4 == 0
        P.sj_specialize(P.SJ_LTIMES, layout="ZDG", variant=P.SJ_VAR_MFMA, tile_n=4,
                        **dict(base, G=6))
    assert e.value.status == P.SJ_ERR_INVALID_ARG
    h = P.sj_specialize(P.SJ_LTIMES, layout="DGZ", dtype=P.SJ_BF16X3, **base)
    assert P.sj_handle_info(h)["kernel_name"] == "sj_ltimes_bf16x3w_dgz"
    h = P.sj_specialize(P.SJ_LTIMES, layout="DGZ", dtype=P.SJ_BF16, tile_n=1, **base)
    assert P.sj_handle_info(h)["kernel_name"] == "sj_ltimes_bf16_dgz"
    with pytest.raises(P.SJError) as e:
        P.sj_specialize(P.SJ_LTIMES, layout="ZDG", dtype=P.SJ_BF16, tile_n=4, **dict(base, G=6))
    assert e.value.status == P.SJ_ERR_INVALID_ARG


def test_bgemm_prefetch_form(P):
    src1 = P.sj_emit_source(P.SJ_BGEMM, order=1)
    src2 = P.sj_emit_source(P.SJ_BGEMM)           # prefetching is the default
    assert "#define SJ_PREFETCH 0" in src1 and "#define SJ_PREFETCH 1" in src2
    h1 = P.sj_specialize(P.SJ_BGEMM, order=1, flags=P.SJ_FLAG_COMPILE_ONLY)
    h2 = P.sj_specialize(P.SJ_BGEMM, order=2, flags=P.SJ_FLAG_COMPILE_ONLY)
    assert h2 == P.sj_specialize(P.SJ_BGEMM, flags=P.SJ_FLAG_COMPILE_ONLY)
    assert h1 != h2 and P.sj_handle_info(h2)["scratch_bytes"] == 0
    with pytest.raises(P.SJError) as e:
        P.sj_specialize(P.SJ_BGEMM, tile_n=7169, flags=P.SJ_FLAG_COMPILE_ONLY)
    assert e.value.status == P.SJ_ERR_INVALID_ARG


def test_load_store_policy_flags(P):
    """The streamed-operand policy: the structure's default, or explicit
    flags for loads and for stores, which are part of the key; the two flags
    of a pair exclude each other."""
    base = dict(Z=4096, G=8, D=48, NM=16)
    co = P.SJ_FLAG_COMPILE_ONLY

    def src(layout, flags=0, **kw):
        return P.sj_emit_source(P.SJ_LTIMES, layout=layout, flags=co | flags, **dict(base, **kw))
    rows = src("ZGD", variant=P.SJ_VAR_MFMA, order=1)
    assert "#define SJ_NT_LOAD 0" in rows and "#define SJ_NT_STORE 1" in rows
    runs = src("ZGD", variant=P.SJ_VAR_MFMA)      # LDS-staged row kernel: whole lines per load
    assert "rows_mfma_lds" in runs and "#define SJ_NT_LOAD 1" in runs and "#define SJ_NT_STORE 1" in runs
    lplus_runs = P.sj_emit_source(P.SJ_LPLUSTIMES, layout="ZGD", flags=co, **base)
    assert "rows_mfma_lds" in lplus_runs and "#define SJ_NT_LOAD 0" in lplus_runs
    cols = src("DGZ")
    assert "#define SJ_NT_LOAD 1" in cols and "#define SJ_NT_STORE 1" in cols
    lplus = P.sj_emit_source(P.SJ_LPLUSTIMES, layout="DGZ", flags=co, **base)
    assert "#define SJ_NT_LOAD 0" in lplus and "#define SJ_NT_STORE 1" in lplus
    mixed = src("DGZ", P.SJ_FLAG_STORES_CACHED)
    assert "#define SJ_NT_LOAD 1" in mixed and "#define SJ_NT_STORE 0" in mixed
    mixed = src("ZGD", P.SJ_FLAG_LOADS_NONTEMPORAL | P.SJ_FLAG_STORES_CACHED, variant=P.SJ_VAR_MFMA, order=1)
    assert "#define SJ_NT_LOAD 1" in mixed and "#define SJ_NT_STORE 0" in mixed
    h0 = P.sj_specialize(P.SJ_LTIMES, layout="DGZ", flags=co, **base)
    h1 = P.sj_specialize(P.SJ_LTIMES, layout="DGZ", flags=co | P.SJ_FLAG_STORES_CACHED, **base)
    assert h0 != h1
    for bad in (P.SJ_FLAG_LOADS_CACHED | P.SJ_FLAG_LOADS_NONTEMPORAL,
                P.SJ_FLAG_STORES_CACHED | P.SJ_FLAG_STORES_NONTEMPORAL):
        with pytest.raises(P.SJError) as e:
            P.sj_specialize(P.SJ_LTIMES, layout="DGZ", flags=co | bad, **base)
        assert e.value.status == P.SJ_ERR_INVALID_ARG


def test_fused_structures(P):
    """LTimes followed by LPlusTimes in one kernel: DIRECT for a column axis
    innermost, the matrix-core row structure for D innermost, DIRECT again
    where the row structure's LDS limit declines the shape; STAGED, the column
    MFMA structure and accumulation are refused."""
    co = P.SJ_FLAG_COMPILE_ONLY

    def name(layout, **kw):
        h = P.sj_specialize(P.SJ_LTIMES_LPLUS, layout=layout, flags=co | kw.pop("flags", 0), **kw)
        return P.sj_handle_info(h)["kernel_name"]
    base = dict(Z=64, G=8, D=96, NM=16)
    assert name("DGZ", **base) == "sj_ltimes_lplus_direct_dgz"
    assert name("ZGD", **base) == "sj_ltimes_lplus_rows_mfma_lds_zgd"
    assert name("ZGD", order=1, **base) == "sj_ltimes_lplus_rows_mfma_zgd"
    assert name("ZGD", Z=64, G=8, D=95, NM=16) == "sj_ltimes_lplus_rows_mfma_zgd"   # odd D: direct operand reads
    assert name("GZD", variant=P.SJ_VAR_DIRECT, **base) == "sj_ltimes_lplus_direct_gzd"
    # 2 x 13 x 4 x 4 weight fragments of 512 bytes exceed the LDS: the next structure takes it
    assert name("ZGD", Z=64, G=8, D=200, NM=49) == "sj_ltimes_lplus_direct_zgd"
    src = P.sj_emit_source(P.SJ_LTIMES_LPLUS, layout="ZGD", flags=co, **base)
    assert "#define SJ_NT_LOAD 1" in src and "#define SJ_NT_STORE 1" in src and "#define SJ_RT 1" in src
    for bad, status in ((dict(layout="ZGD", variant=P.SJ_VAR_STAGED), P.SJ_ERR_UNSUPPORTED),
                        (dict(layout="DGZ", variant=P.SJ_VAR_MFMA), P.SJ_ERR_UNSUPPORTED),
                        (dict(layout="ZGD", variant=P.SJ_VAR_MFMA, D=200, NM=49), P.SJ_ERR_UNSUPPORTED),
                        (dict(layout="ZGD", variant=P.SJ_VAR_MFMA, tile_n=9), P.SJ_ERR_INVALID_ARG),
                        (dict(layout="ZGD", variant=P.SJ_VAR_MFMA, unroll=2), P.SJ_ERR_INVALID_ARG),
                        (dict(layout="ZGD", flags=P.SJ_FLAG_ACCUMULATE), P.SJ_ERR_INVALID_ARG),
                        (dict(layout="ZGD", dtype=P.SJ_BF16), P.SJ_ERR_UNSUPPORTED)):
        spec = dict(base, **bad)
        spec["flags"] = co | spec.get("flags", 0)
        with pytest.raises(P.SJError) as e:
            P.sj_specialize(P.SJ_LTIMES_LPLUS, **spec)
        assert e.value.status == status, bad


def test_values_specs(P):
    """Value specialization: argument checks, the weights as exact literals in
    the emitted code, one compile per distinct value set."""
    import numpy as np
    co = P.SJ_FLAG_COMPILE_ONLY
    base = dict(layout="DGZ", Z=64, G=2, D=8, NM=4, flags=co)
    L = np.arange(32, dtype=np.float64) / 3.0
    s0 = P.sj_stats()
    h1 = P.sj_specialize_values(P.SJ_LTIMES, L, **base)
    h2 = P.sj_specialize_values(P.SJ_LTIMES, L.copy(), **base)
    assert h1 == h2
    assert P.sj_stats()["compiles"] - s0["compiles"] == 1
    assert P.sj_handle_info(h1)["kernel_name"] == "sj_ltimes_direct_values_dgz"
    onehot = np.zeros((4, 8))
    onehot[np.arange(4), [0, 2, 4, 6]] = 1.0
    h3 = P.sj_specialize_values(P.SJ_LTIMES, onehot, **base)
    assert h3 != h1 and P.sj_handle_info(h3)["code_bytes"] < P.sj_handle_info(h1)["code_bytes"]
    bad = [
        (dict(weights=L[:31]), P.SJ_ERR_INVALID_ARG),
        (dict(weights=np.where(np.arange(32) == 3, np.inf, L)), P.SJ_ERR_INVALID_ARG),
        (dict(weights=L, order=2), P.SJ_ERR_INVALID_ARG),
        (dict(weights=L, variant=P.SJ_VAR_MFMA), P.SJ_ERR_UNSUPPORTED),
        (dict(weights=L, kernel=P.SJ_LTIMES_LPLUS), P.SJ_ERR_UNSUPPORTED),
        (dict(weights=np.zeros(4096 * 4), D=4096), P.SJ_ERR_UNSUPPORTED),
    ]
    for b, status in bad:
        b = dict(b)
        kern = b.pop("kernel", P.SJ_LTIMES)
        w = b.pop("weights")
        spec = dict(base, **b)
        with pytest.raises(P.SJError) as e:
            P.sj_specialize_values(kern, w, **spec)
        assert e.value.status == status, b


def test_scattering_specs(P):
    co = P.SJ_FLAG_COMPILE_ONLY
    base = dict(layout="ZGD", Z=40, G=6, NM=9, count=2, flags=co)
    h = P.sj_specialize(P.SJ_SCATTERING, **base)
    assert P.sj_handle_info(h)["kernel_name"] == "sj_scattering_direct_zgd"
    assert h != P.sj_specialize(P.SJ_SCATTERING, **dict(base, count=3))   # the material count is part of the key
    src = P.sj_emit_source(P.SJ_SCATTERING, **base)
    assert "#define SJ_NL 3" in src and "#define SJ_LANE_NM 1" in src and "#define SJ_SG 9" in src
    assert "#define SJ_LANE_NM 0" in P.sj_emit_source(P.SJ_SCATTERING, **dict(base, layout="DGZ",
                                                                               variant=P.SJ_VAR_DIRECT))
    # the vector-FMA structure in ZDG: threads along z by default, along nm (staged degree
    # matrices) with order 2
    zdg = dict(base, layout="ZDG", flags=0, variant=P.SJ_VAR_DIRECT)
    src = P.sj_emit_source(P.SJ_SCATTERING, **zdg)
    assert "#define SJ_LANE_NM 0" in src and "#define SJ_SLDS 0" in src and "#define SJ_RUN_LINES 1" in src
    assert "#define SJ_PERSIST 1" in src   # persistent waves prefetching their next 64 lines
    src = P.sj_emit_source(P.SJ_SCATTERING, **dict(zdg, order=2))
    assert "#define SJ_LANE_NM 1" in src and "#define SJ_SLDS 1" in src and "#define SJ_RUN_LINES 1" in src
    assert "#define SJ_PERSIST 0" in src   # workgroup barriers of the staged matrices: not persistent
    assert "#define SJ_PERSIST 1" in P.sj_emit_source(P.SJ_SCATTERING, **dict(zdg, layout="DZG"))
    assert "#define SJ_PERSIST 0" in P.sj_emit_source(P.SJ_SCATTERING, **dict(zdg, layout="DGZ"))
    # nm fastest with staged degree matrices: two zones per thread
    for lay, pair in (("GZD", 1), ("ZGD", 1), ("DGZ", 0), ("ZDG", 0)):
        assert ("#define SJ_PAIR %d" % pair) in P.sj_emit_source(P.SJ_SCATTERING, **dict(zdg, layout=lay)), lay
    assert P.sj_specialize(P.SJ_SCATTERING, **dict(zdg, flags=co)) != P.sj_specialize(P.SJ_SCATTERING, **dict(zdg, flags=co, order=2))
    # order only changes ZDG: elsewhere 0, 1 and 2 give the same key
    assert len({P.sj_specialize(P.SJ_SCATTERING, **dict(base, order=o)) for o in (0, 1, 2)}) == 1
    for bad, status in ((dict(count=0), P.SJ_ERR_INVALID_ARG), (dict(G=65), P.SJ_ERR_UNSUPPORTED),
                        (dict(variant=P.SJ_VAR_MFMA, G=33), P.SJ_ERR_UNSUPPORTED), (dict(tile_n=2), P.SJ_ERR_INVALID_ARG),
                        (dict(flags=co | P.SJ_FLAG_ACCUMULATE), P.SJ_ERR_INVALID_ARG), (dict(dtype=P.SJ_BF16), P.SJ_ERR_INVALID_ARG),
                        (dict(layout=7), P.SJ_ERR_INVALID_ARG),
                        (dict(order=3), P.SJ_ERR_INVALID_ARG),
                        (dict(layout="ZDG", Z=32768, G=32, NM=16, count=4, block=512, order=2,
                              variant=P.SJ_VAR_DIRECT), P.SJ_ERR_UNSUPPORTED)):
        with pytest.raises(P.SJError) as e:
            P.sj_specialize(P.SJ_SCATTERING, **dict(base, **bad))
        assert e.value.status == status, bad
    # the matrix-core structure where g or z is innermost: tiles per group 1, 2 or 4 (default 2,
    # 1 with zone blocks outer), G <= 32; the default structure there
    mf = dict(base, layout="DZG", variant=P.SJ_VAR_MFMA)
    h = P.sj_specialize(P.SJ_SCATTERING, **mf)
    info = P.sj_handle_info(h)
    assert info["kernel_name"] == "sj_scattering_mfma_dzg" and info["tile_n"] == 2 and info["block"] == 256
    assert P.sj_specialize(P.SJ_SCATTERING, **dict(mf, variant=P.SJ_VAR_AUTO)) == h
    zi = P.sj_handle_info(P.sj_specialize(P.SJ_SCATTERING, **dict(mf, layout="ZDG")))
    assert zi["tile_n"] == 1 and zi["block"] == 128
    assert P.sj_handle_info(P.sj_specialize(P.SJ_SCATTERING, **dict(mf, layout="ZDG", tile_n=4)))["tile_n"] == 4
    for lay in ("DGZ", "GDZ"):
        ci = P.sj_handle_info(P.sj_specialize(P.SJ_SCATTERING, **dict(base, layout=lay)))
        assert ci["kernel_name"] == "sj_scattering_mfma_" + lay.lower() and ci["block"] == 512, lay
    # 64-bit indexing when the matrices alone pass 2^31 elements (65536 materials x 64 degrees x 32^2),
    # though phi is small
    for var in (P.SJ_VAR_AUTO, P.SJ_VAR_DIRECT):
        big = dict(base, layout="DZG", Z=16, G=32, NM=4096, count=65536, variant=var)
        assert "typedef long long sj_index_t" in P.sj_emit_source(P.SJ_SCATTERING, **big), var
        assert "typedef int sj_index_t" in P.sj_emit_source(P.SJ_SCATTERING, **dict(big, count=1)), var
    # G above 32: the vector-FMA structure by default, the matrix cores refused
    assert P.sj_handle_info(P.sj_specialize(P.SJ_SCATTERING, **dict(base, layout="DZG", G=33)))["kernel_name"] == \
        "sj_scattering_direct_dzg"
    src = P.sj_emit_source(P.SJ_SCATTERING, **dict(mf, layout="ZDG"))
    assert "#define SJ_SNM 6" in src and "#define SJ_SZ 54" in src and "#define SJ_RT 1" in src
    assert "#define SJ_ZMAJOR 1" in src   # ZDG: zone blocks outer by default
    assert "#define SJ_ZMAJOR 0" in P.sj_emit_source(P.SJ_SCATTERING, **mf)
    assert "#define SJ_ZMAJOR 1" in P.sj_emit_source(P.SJ_SCATTERING, **dict(mf, order=2))
    # nm innermost: the block form on request (the vector form stays the default there)
    for lay in ("GZD", "ZGD"):
        assert P.sj_handle_info(P.sj_specialize(P.SJ_SCATTERING, **dict(mf, layout=lay)))["kernel_name"] == \
            "sj_scattering_mfma_" + lay.lower()
        assert P.sj_handle_info(P.sj_specialize(P.SJ_SCATTERING, **dict(base, layout=lay)))["kernel_name"] == \
            "sj_scattering_direct_" + lay.lower()
        assert ("#define SJ_ZOUTER %d" % (lay == "ZGD")) in P.sj_emit_source(P.SJ_SCATTERING, **dict(mf, layout=lay))
    # z innermost: the column form (no LDS rows)
    for lay in ("DGZ", "GDZ"):
        src = P.sj_emit_source(P.SJ_SCATTERING, **dict(mf, layout=lay))
        assert "sj_scattering_mfma_" + lay.lower() in src and "__shared__" not in src, lay
    for bad, status in ((dict(tile_n=3), P.SJ_ERR_INVALID_ARG), (dict(G=33), P.SJ_ERR_UNSUPPORTED),
                        (dict(order=3), P.SJ_ERR_INVALID_ARG), (dict(layout="GZD", tile_n=2), P.SJ_ERR_INVALID_ARG),
                        (dict(layout="ZGD", order=2), P.SJ_ERR_INVALID_ARG),
                        (dict(layout="ZGD", G=32, NM=64), P.SJ_ERR_UNSUPPORTED),   # the 16-zone block exceeds LDS
                        (dict(tile_k=8), P.SJ_ERR_INVALID_ARG), (dict(block=1024, tile_n=4, G=32), P.SJ_ERR_UNSUPPORTED)):
        with pytest.raises(P.SJError) as e:
            P.sj_specialize(P.SJ_SCATTERING, **dict(mf, **bad))
        assert e.value.status == status, bad


def test_mass_specs(P):
    co = P.SJ_FLAG_COMPILE_ONLY
    base = dict(D=4, NM=6, inputs=3, count=1000, flags=co)
    h = P.sj_specialize(P.SJ_MASS, **base)
    # default: the pipelined form, four hexahedra per group, 64-thread workgroups
    assert P.sj_handle_info(h)["kernel_name"] == "sj_mass_pa_pipe_3d_d4_q6"
    r = P.sj_resolve(P.SJ_MASS, **base)
    assert (r["order"], r["tile_n"], r["block"]) == (2, 4, 64)
    h1 = P.sj_specialize(P.SJ_MASS, **dict(base, order=1))
    assert P.sj_handle_info(h1)["kernel_name"] == "sj_mass_pa_3d_d4_q6"
    # large elements: the staged form (the pipelined one would hold too many registers)
    assert P.sj_resolve(P.SJ_MASS, **dict(base, D=12, NM=12))["order"] == 1
    src = P.sj_emit_source(P.SJ_MASS, **base)
    assert "#define SJ_DIM 3" in src and "#define SJ_D1D 4" in src and "#define SJ_Q1D 6" in src
    for bad, status in ((dict(inputs=4), P.SJ_ERR_INVALID_ARG), (dict(D=33), P.SJ_ERR_INVALID_ARG),
                        (dict(count=0), P.SJ_ERR_INVALID_ARG), (dict(variant=P.SJ_VAR_MFMA), P.SJ_ERR_UNSUPPORTED),
                        (dict(unroll=2), P.SJ_ERR_INVALID_ARG), (dict(D=32, NM=32, block=1024), P.SJ_ERR_UNSUPPORTED),
                        (dict(dtype=P.SJ_F32), P.SJ_ERR_INVALID_ARG)):
        with pytest.raises(P.SJError) as e:
            P.sj_specialize(P.SJ_MASS, **dict(base, **bad))
        assert e.value.status == status, bad


def test_bf16_wide_block_limit(P):
    """Four columns per lane need at most 512 threads per block (1024 would spill)."""
    co = P.SJ_FLAG_COMPILE_ONLY
    with pytest.raises(P.SJError) as e:
        P.sj_specialize(P.SJ_LTIMES, layout="DGZ", Z=4096, G=8, D=48, NM=16, dtype=P.SJ_BF16X3, tile_n=4, block=1024,
                        flags=co)
    assert e.value.status == P.SJ_ERR_UNSUPPORTED
    P.sj_specialize(P.SJ_LTIMES, layout="DGZ", Z=4096, G=8, D=48, NM=16, dtype=P.SJ_BF16X3, tile_n=4, block=512, flags=co)
