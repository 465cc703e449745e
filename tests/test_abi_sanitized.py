"""The C-ABI tests (tests/test_abi.py: symbols, argument validation, limits,
no device work) against a build of the library whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer, in a child process with the
sanitizer runtime preloaded.  Any sanitizer report fails the test.  CPU only;
the sanitized build (about a minute) is made here when it is missing or older
than the sources."""
import os
import subprocess
import sys

import pytest

from paper_1706_06972_amd import build as Bld

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1706_06972_amd", "csrc")


def stale() -> bool:
    if not os.path.exists(Bld.LIB_SANITIZED):
        return True
    t = os.path.getmtime(Bld.LIB_SANITIZED)
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(ROOT, "include", "ocsc.h")]
    return any(os.path.getmtime(f) > t for f in srcs)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_abi_under_address_and_undefined_behaviour_sanitizers():
    if stale():
        Bld.build_sanitized()
    env = dict(os.environ)
    env["OCSC_LIBRARY"] = Bld.LIB_SANITIZED
    env["LD_PRELOAD"] = Bld.asan_runtime()
    # the interpreter itself is not instrumented: leak reports would list its own allocations
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-3000:]
    assert r.returncode == 0, out[-3000:]
    assert " passed" in out
