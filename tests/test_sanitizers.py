"""CPU: the host side under AddressSanitizer and UndefinedBehaviorSanitizer.

The diagram compiler and the host logic of the library (libdd_san.so: host objects built with
-fsanitize=address,undefined, device code as usual) and the FP64 oracle (liboracle_san.so) are
rebuilt with the sanitizers, and the host and oracle tests run against them in a child process
that preloads gcc's sanitizer runtimes, halting on the first report.  No GPU is used: device code
is never reached on this path."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_host_code_and_oracle_under_asan_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not found")
    from paper_2205_11638_amd import build as b
    b.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", DD_SANITIZE="1", ORACLE_SANITIZE="1",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    subprocess.check_call([sys.executable, "-c", "from oracle import oracle; oracle.build(force=True)"], cwd=ROOT,
                          env={k: v for k, v in env.items() if k != "LD_PRELOAD"})
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_host.py", "tests/test_oracle_pins.py", "-q", "-x",
                        "-m", "not gpu", "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
