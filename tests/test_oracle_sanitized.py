"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's source is built with -fsanitize=address,undefined (UB aborts) and
the oracle pin suites run against that build, loaded into the interpreter with
the sanitizer runtimes preloaded.  A control build with a planted out-of-bounds
read must abort with an AddressSanitizer report, which shows the instrumented
build is the one loaded.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rlb_oracle.cpp")
PINS = [os.path.join(ROOT, "tests", f) for f in
        ("test_oracle_pins.py", "test_oracle_positivity.py", "test_oracle_eos.py",
         "test_oracle_transport.py", "test_oracle_gradients.py", "test_oracle_riemann.py")]
FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fPIC",
         "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def _runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


ASAN, UBSAN = _runtime("libasan.so"), _runtime("libubsan.so")
pytestmark = pytest.mark.skipif(not (ASAN and UBSAN), reason="sanitizer runtimes not installed")


def _build(src_text, out):
    src = out + ".cpp"
    with open(src, "w") as fh:
        fh.write(src_text)
    subprocess.run(["g++", *FLAGS, "-o", out, src], check=True, capture_output=True)


def _run_pins(lib, files, log=None):
    """The pin files against the sanitized build; reports go to log.<pid> when
    log is given (pytest's own capture would swallow them on abort)."""
    asan = "detect_leaks=0:abort_on_error=1" + (f":log_path={log}" if log else "")
    ubsan = "print_stacktrace=1:halt_on_error=1" + (f":log_path={log}" if log else "")
    env = dict(os.environ, RLB_ORACLE_LIB=lib, LD_PRELOAD=f"{ASAN}:{UBSAN}",
               ASAN_OPTIONS=asan, UBSAN_OPTIONS=ubsan)
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           *files], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)


def test_pin_suites_pass_under_address_and_ub_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    _build(open(SRC).read(), lib)
    r = _run_pins(lib, PINS)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])


def test_sanitizer_catches_a_planted_out_of_bounds_read(tmp_path):
    src = open(SRC).read()
    old = "long si = L.index(b, s[0], s[1], s[2]);"
    assert src.count(old) == 1
    lib = str(tmp_path / "liboracle_oob.so")
    _build(src.replace(old, "long si = L.index(b, s[0], s[1], s[2]) + L.cells();"), lib)
    log = str(tmp_path / "asan")
    r = _run_pins(lib, [PINS[0]], log=log)
    assert r.returncode != 0
    reports = [open(os.path.join(tmp_path, f)).read() for f in os.listdir(tmp_path)
               if f.startswith("asan.")]
    assert any("AddressSanitizer" in t for t in reports), (r.stdout[-2000:], r.stderr[-2000:])
