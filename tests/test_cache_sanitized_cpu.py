"""The specialization cache under concurrent requests (compile-only keys, no
GPU): 8 threads request 6 keys and one failing key in shuffled orders while a
reader polls the statistics.  Each key must compile once and yield one handle
in every thread; the failing key must reach every requester and never stay in
the cache.  Run on the plain build and on builds whose host code (library and
program) is instrumented by ThreadSanitizer and by AddressSanitizer (with leak
detection): no report may appear."""
import json
import os
import subprocess

import pytest

from paper_1904_08555_amd import build as B


def run_stress(exe, env=None):
    r = subprocess.run([exe, "8", "3"], capture_output=True, text=True, timeout=300, env=env)
    out = json.loads(r.stdout.strip().splitlines()[-1])
    return r, out


def test_cache_stress_plain():
    exe = B.build_cache_stress()
    r, out = run_stress(exe)
    assert r.returncode == 0 and out["ok"], (out, r.stderr[-2000:])
    assert out["entries"] == 6 and out["same_handles"] and out["failed_requests"] == 24


@pytest.mark.parametrize("kind", ["thread", "address"])
def test_cache_stress_sanitized(kind, tmp_path):
    exe = B.build_sanitized(kind, str(tmp_path / kind))
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 second_deadlock_stack=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    r, out = run_stress(exe, env)
    assert "ThreadSanitizer" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "LeakSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and out["ok"], (out, r.stderr[-2000:])
