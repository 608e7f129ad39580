"""Host-only native tests (no GPU): the request server's admission rule, and a
sanitizer build (AddressSanitizer + UndefinedBehaviorSanitizer) of the einsum
parser and the oracle.  Built with the host compilers only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2206_08301_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (" ".join(cmd)) + "\n" + r.stdout + r.stderr
    return r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_admission_rule(tmp_path):
    exe = str(tmp_path / "sched")
    _run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, os.path.join(NATIVE, "sched_driver.cpp"), "-o", exe],
         str(tmp_path))
    out = _run([exe], str(tmp_path))
    assert "sched: ok" in out


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="needs gcc and g++")
def test_parser_and_oracle_under_sanitizers(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    inc = ["-I", CSRC, "-I", os.path.join(ROOT, "include")]
    objs = []
    for src, lang in ((os.path.join(CSRC, "parse.cpp"), "c++"), (os.path.join(CSRC, "errors.cpp"), "c++"),
                      (os.path.join(NATIVE, "san_driver.cpp"), "c++")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run(["g++", "-std=c++17", *san, *inc, "-c", src, "-o", obj], str(tmp_path))
        objs.append(obj)
    oobj = str(tmp_path / "oracle.o")
    _run(["gcc", "-std=c11", *san, "-fopenmp", "-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o", oobj],
         str(tmp_path))
    exe = str(tmp_path / "san")
    _run(["g++", *san, "-fopenmp", *objs, oobj, "-o", exe], str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], cwd=str(tmp_path), capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "san: accepted" in r.stdout and "ERROR" not in r.stderr
