"""The oracle and the library's host validation layer built for the CPU
with AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only;
no GPU code is built here), then run over valid and malformed inputs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_and_host_checks_under_sanitizers(tmp_path):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("no host compiler")
    exe = str(tmp_path / "driver")
    objs = []
    for src, cc in [(os.path.join(ROOT, "oracle", "oracle.c"), "gcc"),
                    (os.path.join(ROOT, "paper_2609_07204_amd", "csrc", "mc_host.cpp"), "g++"),
                    (os.path.join(ROOT, "tests", "sanitize", "driver.cpp"), "g++")]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [cc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-I" + os.path.join(ROOT, "include"), "-c", src, "-o", obj]
        if cc == "g++":
            cmd.insert(1, "-std=c++17")
        subprocess.run(cmd, check=True)
        objs.append(obj)
    subprocess.run(["g++", "-fsanitize=address,undefined"] + objs + ["-o", exe], check=True)
    # a library preloaded by the environment may come before the ASan
    # runtime; ASan's own option accepts that order
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env, timeout=300)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "sanitize driver ok" in p.stdout
    assert "runtime error" not in p.stderr
