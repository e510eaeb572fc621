"""Sanitizer builds of the host-side code (CPU only).

The C oracles (oracle/lbm3_oracle.c, oracle/lbm3_oracle3d.c) are built with gcc and the
address and undefined-behaviour sanitizers (leak checks on) and driven through every entry
point on small and degenerate lattices, every segregation law and both forcings
(tests/sanitize/oracle_main.c).  The library's sources are built with hipcc with the same
sanitizers on the host side only, and a driver (tests/sanitize/host_main.cpp) runs its
host code: parameter validation and derived constants over valid and invalid inputs,
density checks, tile plans (every node in exactly one tile) with their XCD ordering and row
choice, and the adjoint's slot rule.  Any report aborts the driver."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", os.path.join(HERE, "oracle_main.c"),
          os.path.join(ROOT, "oracle", "lbm3_oracle.c"), os.path.join(ROOT, "oracle", "lbm3_oracle3d.c"),
          "-lm", "-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert r.stdout.strip() == "ok"


def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1808_08555_amd import build as B
    if not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-g"]
    srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES] + [os.path.join(HERE, "host_main.cpp")]
    procs, objs = [], []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        flags = list(B.CFLAGS)
        for extra in B.PER_FILE.get(os.path.basename(src), []):
            key = extra.split("=")[0]
            flags = [f for f in flags if f.split("=")[0] != key] + [extra]
        procs.append(subprocess.Popen([B.HIPCC, *flags, *san, "-I", B.CSRC, "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    for p, src in zip(procs, srcs):
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, f"{src}\n{err[-3000:]}"
    exe = str(tmp_path / "host_san")
    _run(["g++", "-fsanitize=address,undefined", *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert r.stdout.strip() == "ok"
