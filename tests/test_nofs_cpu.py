"""The specialization library reads no file (ClangJIT sections 1 and 4: an
instantiation uses only what the running binary holds; nothing is read from
or written to a file by the library itself).

A child process loads a copy of ``libsj.so`` placed alone in an empty
directory, away from the source tree and its kernel templates, with the open
probe of ``fsprobe/fsprobe.c`` preloaded.  Recording is switched on around
one specialization miss (compile only: no GPU is needed) and every file open
during it is attributed to the shared object that asked for it.  The test
asserts that:
  * the miss succeeds, so the kernel templates come from the library binary;
  * no open is charged to libsj itself;
  * the probe works (a positive control: a file the child opens on purpose
    while recording is in the log).
Opens charged to the compiler (hiprtc and the code-object manager it drives,
which stages temporaries of its own under the temporary directory) are the
known exception: they are reported, not failed.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE_SRC = os.path.join(ROOT, "tests", "fsprobe", "fsprobe.c")

CHILD = textwrap.dedent("""
    import ctypes, os, sys
    sys.path.insert(0, sys.argv[1])
    import paper_1904_08555_amd.sj as sj
    sj.LIB_PATH = sys.argv[2]
    lib = sj.lib()
    probe = ctypes.CDLL(None)
    # a first miss loads and initialises the compiler; the recorded one is the second
    sj.sj_specialize(sj.SJ_LTIMES, layout="ZGD", Z=31, G=3, D=10, NM=4, flags=sj.SJ_FLAG_COMPILE_ONLY)
    probe.fsprobe_enable(1)
    h = sj.sj_specialize(sj.SJ_LTIMES, layout="DZG", Z=53, G=7, D=11, NM=5, flags=sj.SJ_FLAG_COMPILE_ONLY)
    with open(sys.argv[3], "w") as f:       # positive control
        f.write("x")
    probe.fsprobe_enable(0)
    assert h, "no handle"
    print("CHILD_OK", flush=True)
""")


@pytest.fixture(scope="module")
def probe_so(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is needed to build the open probe")
    d = tmp_path_factory.mktemp("fsprobe")
    so = str(d / "fsprobe.so")
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-o", so, PROBE_SRC, "-ldl"], check=True)
    return so


def test_library_opens_no_file_on_a_miss(probe_so, tmp_path):
    import paper_1904_08555_amd as P
    P.lib()                                  # built
    alone = tmp_path / "alone"
    alone.mkdir()
    lib_copy = str(alone / "libsj.so")
    shutil.copy(P.sj.LIB_PATH, lib_copy)     # no kernel templates beside it
    log = str(tmp_path / "opens.tsv")
    control = str(tmp_path / "control.txt")
    env = dict(os.environ)
    env["FSPROBE_LOG"] = log
    env["LD_PRELOAD"] = probe_so + ((" " + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, lib_copy, control], cwd=str(alone), env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "CHILD_OK" in r.stdout, r.stdout + r.stderr
    rows = []
    with open(log) as f:
        for line in f:
            fn, path, who = line.rstrip("\n").split("\t")
            rows.append((fn, path, who))
    assert any(p == control for _, p, _ in rows), f"probe recorded nothing useful: {rows[:10]}"
    own = [r for r in rows if os.path.basename(r[2]).startswith("libsj")]
    assert not own, f"libsj opened files during a specialization miss: {own}"
    others = sorted({(os.path.basename(w), os.path.dirname(p)) for _, p, w in rows if p != control})
    # whatever else opened files is the compiler and its code-object manager
    for who, _ in others:
        assert "libsj" not in who
    print("opens by other objects during the miss:", others)
