"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
library's family builder (family.cpp) and the CPU reference
(oracle/pd_oracle.c) built with g++/gcc -fsanitize=address,undefined and run
by tests/sanitize/driver.cpp on small workloads of every kind (3D box,
notched plates, three specimens, a wide horizon, the double-notched 3D
plate, the notched cylinder) through every host entry point; any finding
aborts the driver."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_host_code_is_clean_under_sanitizers(tmp_path):
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2309_11273_amd", "csrc")]
    objs = []
    for src, cc, std in ((os.path.join(ROOT, "paper_2309_11273_amd", "csrc", "family.cpp"), "g++", "-std=c++17"),
                         (os.path.join(ROOT, "oracle", "pd_oracle.c"), "gcc", "-std=c11"),
                         (os.path.join(ROOT, "tests", "sanitize", "driver.cpp"), "g++", "-std=c++17")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        extra = ["-ffp-contract=off"] if src.endswith(".c") else ["-pthread"]
        subprocess.check_call([cc, std, "-c", src, "-o", obj] + SAN + inc + extra)
        objs.append(obj)
    exe = str(tmp_path / "sanitize_driver")
    subprocess.check_call(["g++", "-o", exe] + objs + SAN + ["-static-libasan", "-pthread", "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitize: ok" in r.stdout
