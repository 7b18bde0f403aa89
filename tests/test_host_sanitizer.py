"""The library's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer (CPU only): the host-sanitizer build (build.py: the ABI, request
server, allocator and host numerics instrumented on their host pass, device
code as usual) runs the host-only ABI tests in a child process, with the
sanitizer runtime preloaded ahead of whatever the environment preloads.  Any
report ends that process with an error."""
import os
import subprocess
import sys

from paper_2202_11288_amd import build as BLD

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_abi_cpu.py", "tests/test_abi_standard_cpu.py",
              "tests/test_abi_shift_cpu.py", "tests/test_abi_ws_cpu.py"]


def test_host_code_under_sanitizers():
    lib = BLD.build_sanitized()
    preload = [BLD.sanitizer_runtime()]
    if os.environ.get("LD_PRELOAD"):
        preload.append(os.environ["LD_PRELOAD"])
    env = dict(os.environ, LD_PRELOAD=":".join(preload), AMG_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *HOST_TESTS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-4000:] + "\n" + r.stderr[-4000:])
    assert r.returncode == 0, tail
    assert " passed" in r.stdout and "error" not in r.stdout.lower().split("passed")[-1], tail
