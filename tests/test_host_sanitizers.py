"""The host code of the library under AddressSanitizer and
UndefinedBehaviorSanitizer: the host-only ABI tests (symbols, validation,
layouts, footprints, error paths) run in a child process against the
sanitized build with the sanitizer runtime preloaded; any report fails the
child.  CPU only (no device code runs)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILDER = os.path.join(ROOT, "paper_2411_05510_amd", "build_sanitized.py")


@pytest.mark.skipif(not os.path.exists(BUILDER), reason="sanitized builder not present")
def test_host_abi_under_asan_and_ubsan():
    from paper_2411_05510_amd import build_sanitized as BS
    lib = BS.build()
    env = dict(os.environ)
    env.update({
        "SSI_LIBRARY": lib,
        "LD_PRELOAD": BS.runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    probe = ("import ctypes; from paper_2411_05510_amd import ssicov as S; S.lib(); "
             "maps = open('/proc/self/maps').read(); "
             "assert S.LIB_PATH in maps and 'asan' in maps, 'sanitized build not loaded'")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join("tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
