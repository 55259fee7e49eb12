"""The oracle's C code under UndefinedBehaviorSanitizer (gcc): random machines
with operands over the whole int32 range, both instruction sets, several word
widths, and the hand-traced programs, in a child process that aborts on the
first report."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, os, sys
sys.path.insert(0, {root!r})
import oracle
oracle._LIB_PATH = {lib!r}
oracle._lib = None
from paper_2604_12902_amd import workloads as W
for isa in (0, 1):
    b = W.tiny_random(seed=41 + isa, num_vms=4000, isa=isa, max_m=10, max_n=37,
                      operand_lo=-(1 << 31), operand_hi=(1 << 31) - 1)
    for w in (3, 8, 29, 32):
        oracle.run(b, 300, w=w, threads=2)
with open(os.path.join({root!r}, "tests", "golden", "hand_traces.json")) as f:
    cases = json.load(f)["cases"]
for c in cases:
    isa = W.ISA_CLASSIC if c["isa"] == "classic" else W.ISA_WORD
    b = W.from_programs(isa, [c["words"]], c["n"], [c["tape"]], ell=c["ell"], s=c["s"])
    st = oracle.run(b, c["budget"])
    assert int(st.steps[0]) == c["expect"]["steps"], c["name"]
loaded = [l for l in open("/proc/self/maps").read().splitlines() if l.endswith({lib!r})]
assert loaded, "the sanitized oracle was not loaded"
print("ok")
"""


def test_oracle_runs_clean_under_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    ubsan = subprocess.run([gcc, "-print-file-name=libubsan.so"], capture_output=True,
                           text=True).stdout.strip()
    if not os.path.isabs(ubsan) or not os.path.exists(ubsan):
        pytest.skip("libubsan not available")
    lib = str(tmp_path / "liboracle_ubsan.so")
    subprocess.run([gcc, "-O1", "-std=c11", "-fPIC", "-shared", "-pthread",
                    "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                    "-o", lib, os.path.join(ROOT, "oracle", "rasp_oracle.c")], check=True)
    env = dict(os.environ, LD_PRELOAD=ubsan, UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-3000:]
