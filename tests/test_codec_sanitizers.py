"""The library's host codec (csrc/codec.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer by g++ (host code only) and driven by
tests/codec_fuzz.cpp: random valid and malformed genotypes, encode/decode
round trips and random byte programs through validate, with every
sanitizer report fatal."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_codec_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "codec_fuzz")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2605_30954_amd", "csrc"),
           os.path.join(ROOT, "paper_2605_30954_amd", "csrc", "codec.cpp"),
           os.path.join(ROOT, "tests", "codec_fuzz.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    trips = int(r.stdout.split(",")[1].split()[0])
    assert trips >= 200, r.stdout      # enough valid batches reach the round trip
