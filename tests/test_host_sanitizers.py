"""The host C++ of the library (partition set-up, split checks, column
restriction, general partition, Gramian bases by eigenpairs and by the
Zolotarev projector, corner-set removal, argument validation) under
AddressSanitizer and UndefinedBehaviorSanitizer: the library is rebuilt
with both sanitizers on its host code (build.build_sanitized) and the
host-only ABI tests run against it in a child process with the ASan runtime
preloaded; any report aborts that process (UBSan without recovery)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_abi_under_asan_and_ubsan():
    from paper_1604_06750_amd import build
    rt = build.asan_runtime()
    if not rt or not os.path.exists(rt):
        pytest.skip("ASan runtime not found")
    lib = build.build_sanitized(verbose=False)
    env = dict(os.environ, LD_PRELOAD=rt, SFROM_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    script = (
        "import sys, pytest\n"
        "from paper_1604_06750_amd import sfrom\n"
        f"assert sfrom.LIB_PATH == {lib!r}, sfrom.LIB_PATH\n"
        "maps = open('/proc/self/maps').read()\n"
        "assert 'libclang_rt.asan' in maps and sfrom.LIB_PATH in maps\n"
        "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', 'tests/test_abi_host.py', "
        "'tests/test_abi_general.py', 'tests/test_abi_corners.py']))\n")
    r = subprocess.run([sys.executable, "-c", script], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1500)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
