"""The host-side tests again, under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's host code (planner, field code, C-ABI layer) and the oracle are
rebuilt with -fsanitize=address,undefined (gcc), and tests/test_library_host.py
and tests/test_oracle.py run in a child process with the ASan runtime preloaded
and the sanitized builds loaded in place of the ordinary ones.  Any report
(heap or stack overflow, use after free, signed overflow, misaligned access,
...) fails the test.  A planted overflow in a throw-away library checks that
the harness does detect reports.  (The address-space-limited ENOMEM probe is
left out there: ASan's shadow memory needs an unlimited address space.)
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CONTROL_C = r"""
#include <stdlib.h>
int overflow_once(int i) { int* v = (int*)malloc(4 * sizeof(int)); v[i] = 1; int r = v[0]; free(v); return r; }
"""


def _libasan():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    asan = _libasan()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    sys.path.insert(0, ROOT)
    from paper_2101_01025_amd import build_host_sanitized as bhs
    try:
        bhs.device_objects()
    except FileNotFoundError as e:
        pytest.skip(f"ordinary build missing ({e}); run __graft_entry__.build() first")
    out = tmp_path_factory.mktemp("hostsan")
    lib = bhs.build(str(out))
    olib = str(out / "liboracle_hostsan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                           "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-fno-sanitize-recover=undefined", "-o", olib,
                           os.path.join(ROOT, "oracle", "oracle.c")])
    ctl_src = out / "control.c"
    ctl_src.write_text(CONTROL_C)
    ctl = str(out / "libcontrol.so")
    subprocess.check_call(["gcc", "-O0", "-g", "-shared", "-fPIC", "-fsanitize=address", "-o", ctl,
                           str(ctl_src)])
    env = dict(os.environ)
    env.update(LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               FFA_LIBRARY=lib, ORACLE_LIBRARY=olib)
    return env, lib, olib, ctl


def test_harness_detects_a_planted_overflow(sanitized):
    env, _, _, ctl = sanitized
    code = f"import ctypes; ctypes.CDLL({ctl!r}).overflow_once(4)"
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]


def test_sanitized_builds_are_the_ones_loaded(sanitized):
    env, lib, olib, _ = sanitized
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2101_01025_amd as ffa, oracle\n"
            "ffa.lib(); oracle.lib()\n"
            "maps = open('/proc/self/maps').read()\n"
            "print(all(x in maps for x in (%r, %r, 'libasan')))\n" % (ROOT, lib, olib))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "True", (r.stdout, r.stderr[-2000:])


def test_host_tests_pass_under_sanitizers(sanitized):
    env, _, _, _ = sanitized
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", "not host_allocation_failure",
                        os.path.join(ROOT, "tests", "test_library_host.py"),
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
