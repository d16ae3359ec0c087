"""Host code under AddressSanitizer and UBSan (CPU only; no GPU code is built
this way): the oracle's C library runs the oracle pins, and the serving
loop's scheduler runs random schedules over its simulated executor."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    path = subprocess.run([gcc, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not found")
    return path


def _san_env(**extra):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.update(extra)
    return env


def test_oracle_pins_under_sanitizers(tmp_path):
    """Every pin of the oracle (the planted-mistake runs aside: they test the
    pins, not the oracle) against a build of utf16_oracle.c with
    AddressSanitizer and UBSan loaded into the test process."""
    asan = _runtime("libasan.so")
    so = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-std=c11", *SAN, "-fPIC", "-shared", "-pthread", "-o", str(so),
                    os.path.join(ROOT, "oracle", "utf16_oracle.c")], check=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", "not planted"],
                       cwd=ROOT, capture_output=True, text=True, timeout=600,
                       env=_san_env(LD_PRELOAD=asan, UTF16WF_ORACLE_LIB=str(so)))
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-4000:]
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert " passed" in text


def test_oracle_under_sanitizers_is_the_oracle(tmp_path):
    """The sanitizer build is loaded, not the plain one: a child process that
    loads it through the override reports its path."""
    asan = _runtime("libasan.so")
    so = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-std=c11", *SAN, "-fPIC", "-shared", "-pthread", "-o", str(so),
                    os.path.join(ROOT, "oracle", "utf16_oracle.c")], check=True)
    code = ("import oracle, numpy as np; L = oracle._load(); print(L._name); "
            "s = np.array([0xDC00, 0x41, 0xD800], np.uint16); print(oracle.to_well_formed(s).tolist())")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120,
                       env=_san_env(LD_PRELOAD=asan, UTF16WF_ORACLE_LIB=str(so)))
    assert r.returncode == 0, r.stderr[-2000:]
    lines = r.stdout.split("\n")
    assert lines[0] == str(so)
    assert lines[1] == "[65533, 65, 65533]"


def test_scheduler_under_sanitizers(tmp_path):
    _runtime("libasan.so")
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = tmp_path / "serve_sim_check"
    subprocess.run([gxx, "-std=c++17", *SAN, "-Wall", "-Wextra", "-o", str(exe),
                    os.path.join(ROOT, "tests", "sanitize", "serve_sim_check.cpp")], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=_san_env())
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert r.stdout.strip().endswith("ok")
