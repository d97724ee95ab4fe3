"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

oracle/hepkref.c is compiled with -fsanitize=address,undefined (every
finding fatal) and the oracle's pins (tests/test_oracle_pins.py) run against
that build in a child process: an out-of-bounds access, a use after free or
an undefined operation anywhere the pins reach fails this test.
"""
import os
import subprocess
import sys

import pytest

from oracle import ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc has no AddressSanitizer runtime here")
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "libhepkref_san.so")
    subprocess.check_call(["gcc", *ref.CFLAGS, "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-shared", "-o", lib, ref.SRC, "-lm"])
    env = dict(os.environ)
    env["HEPKREF_LIB"] = lib
    # the sanitizer runtime has to come first among the preloaded libraries
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = _runtime("libasan.so") + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-4000:] + r.stderr[-4000:])
    assert "passed" in r.stdout
