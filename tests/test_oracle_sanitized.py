"""The C++ oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host code only, every report fatal) runs the oracle's CPU pins clean.

The pins run in a child pytest process with the ASan runtime preloaded and
ORQA_ORACLE_LIB pointing at the sanitized build; leak checking is off (the
Python interpreter itself is not built for it).  The 41-second untruncated
t = 5 case of Table 1 is left out (it takes minutes under the sanitizers);
every other oracle pin runs."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _asan_runtime():
    if shutil.which("g++") is None:
        return None
    path = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    import oracle
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("g++ with the ASan runtime is not available")
    lib = oracle.build(out=str(tmp_path / "liborqa_oracle_san.so"), sanitize=True)
    with open(lib, "rb") as f:
        image = f.read()
    assert b"__asan_init" in image and b"__ubsan_handle" in image  # instrumented
    env = dict(os.environ)
    env["ORQA_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = rt + (" " + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    probe = subprocess.run([sys.executable, "-c", "import oracle; oracle._load(); print(oracle._LIB)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0 and probe.stdout.strip() == lib, probe.stdout + probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", "not test_table1_t5_untruncated", "tests/test_oracle_pins.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert r.returncode == 0, out[-4000:]
    assert "passed" in r.stdout
    for bad in ("AddressSanitizer", "runtime error:", "UndefinedBehaviorSanitizer"):
        assert bad not in out, out[-4000:]
