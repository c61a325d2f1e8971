"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs
every fast pin without a report (memory errors or undefined behaviour in the
checker would make its answers meaningless).  A planted out-of-bounds read
(ORACLE_MUTANT=18) must be reported, which shows the sanitizers are live.
The pins run in a child process that preloads the sanitizer runtimes."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r"""
import sys
sys.path.insert(0, {here!r}); sys.path.insert(0, {root!r})
import oracle, oracle_pins as P
o = oracle.Oracle({lib!r})
for pin in P.FAST_PINS:
    pin(o)
print("pins-done", len(P.FAST_PINS), flush=True)
"""


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run(lib):
    env = dict(os.environ)
    env["LD_PRELOAD"] = ":".join([_runtime("libasan.so"), _runtime("libubsan.so")])
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    env["OMP_NUM_THREADS"] = "2"
    code = CHILD.format(here=HERE, root=ROOT, lib=lib)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                          env=env, timeout=600)


@pytest.mark.skipif(_runtime("libasan.so") is None or _runtime("libubsan.so") is None,
                    reason="gcc sanitizer runtimes not installed")
@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_oracle_pins_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        lib = oracle.build(0, out=os.path.join(d, "liboracle_asan.so"), sanitize=True)
        r = _run(lib)
        assert r.returncode == 0 and "pins-done" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
        bad = oracle.build(18, out=os.path.join(d, "liboracle_asan_mut18.so"), sanitize=True)
        r = _run(bad)
        assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stderr[-2000:]
