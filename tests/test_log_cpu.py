"""SJ_LOG=1: the library writes one line per specialization it builds (or
fails to build) to stderr, naming the kernel, the key hash and the emit,
compile and load times; without it, nothing."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROG = """
import paper_1904_08555_amd as P
P.sj_specialize(P.SJ_LTIMES, layout='ZGD', Z=40, G=3, D=12, NM=4, flags=P.SJ_FLAG_COMPILE_ONLY)
P.sj_specialize(P.SJ_LTIMES, layout='ZGD', Z=40, G=3, D=12, NM=4, flags=P.SJ_FLAG_COMPILE_ONLY)   # a hit: no line
try:
    P.sj_specialize(P.SJ_LTIMES, layout='ZGD', Z=40, G=3, D=12, NM=4,
                    flags=P.SJ_FLAG_COMPILE_ONLY | P.SJ_FLAG_DEBUG_FAIL_COMPILE)
except P.SJError:
    pass
"""


def run(env_value):
    env = dict(os.environ)
    env.pop("SJ_LOG", None)
    if env_value is not None:
        env["SJ_LOG"] = env_value
    r = subprocess.run([sys.executable, "-c", PROG], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return [ln for ln in r.stderr.splitlines() if ln.startswith("sj: ")]


def test_log_lines():
    lines = run("1")
    assert len(lines) == 2, lines
    assert lines[0].startswith("sj: built sj_ltimes_") and "compile=" in lines[0] and "key=" in lines[0]
    assert lines[1].startswith("sj: FAILED sj_ltimes_")


def test_log_off():
    assert run(None) == [] and run("0") == []
