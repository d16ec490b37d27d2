"""Host C code under AddressSanitizer and UndefinedBehaviorSanitizer.  First
the oracle's:
tests/sanitize_driver.c (key generation, encryption, decryption, decoding
inside and beyond the radius, Reed-Solomon, the KEM with honest and
tampered ciphertexts, the transform, ring multiplication; all parameter
sets) is built with gcc and every sanitizer report aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "sanitize_driver")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
           os.path.join(ROOT, "tests", "sanitize_driver.c")] + \
          [os.path.join(ROOT, "oracle", f) for f in ("hqc_oracle.c", "kem_oracle.c", "ring_oracle.c")] + \
          ["-lpthread"]
    subprocess.check_call(cmd)
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)  # the sanitizer runtime must come first
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(" ok") == 3


def test_input_generator_under_address_and_undefined_sanitizers(tmp_path):
    """The product package's seeded input generator (csrc/hqc_synth.c, with
    its threads) under the same sanitizers, driven by
    tests/sanitize_synth_driver.c."""
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "sanitize_synth")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
           os.path.join(ROOT, "tests", "sanitize_synth_driver.c"),
           os.path.join(ROOT, "paper_2512_12904_amd", "csrc", "hqc_synth.c"), "-lpthread"]
    subprocess.check_call(cmd)
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(" ok") == 3
