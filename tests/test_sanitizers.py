"""Sanitizer builds of the CPU code (no GPU): the oracle under
AddressSanitizer + UndefinedBehaviorSanitizer through a C driver of its
whole interface, and the C-ABI library's host code (model validation,
flattening, code generation, work accounting) under
UndefinedBehaviorSanitizer.  Any sanitizer report fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1010_2438_amd", "csrc")


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    r = subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                        os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                        os.path.join(ROOT, "oracle", "ssa.c"), "-o", exe, "-lm", "-lpthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.startswith("ok")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


HOST_EXERCISE = r'''
import sys
sys.path.insert(0, sys.argv[2])
import paper_1010_2438_amd.abi as A
A.load(sys.argv[1])
import paper_1010_2438_amd as P
import workloads as W
models = [W.config(i)[0] for i in range(4)] + [
    W.birth_death(), W.isomerisation(), W.pure_decay(), W.dimerisation(), W.paper_example(),
    W.transport(), W.transport(n_children=7), W.receptor_binding(),
    W.multi_compartment(3, n_cells_=1), W.multi_compartment(3, n_cells_=10)]
for m in models:
    P.cwc_model_describe(m)
    assert len(P.cwc_codegen(m)) > 1000
bad = []
b = W.lotka_volterra(); b["rules"][0]["k"] = 0.0; bad.append(b)
b = W.lotka_volterra(); b["rules"][1]["lhs"]["p"] = {0: 2, 1: 1}; bad.append(b)
b = W.lotka_volterra(); b["rules"][0]["lhs"]["p"] = {5: 1}; bad.append(b)
b = W.lotka_volterra(); b["init"] = [[-1, 3]]; bad.append(b)
b = W.transport(); b["compartments"][1]["parent"] = 2; bad.append(b)
b = W.transport(); b["rules"][0]["lhs"] = {"w": {0: 1}}; bad.append(b)
bad.append(W.multi_compartment(3, n_cells_=70))
for b in bad:
    try:
        P.cwc_codegen(b)
        raise SystemExit("accepted a malformed model")
    except P.CwcError:
        pass
print("ok")
'''


def test_library_host_code_under_ubsan(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/"
                          "libclang_rt.ubsan_standalone-x86_64.so"))
    if not rt:
        pytest.skip("no UBSan runtime for the ROCm compiler")
    from paper_1010_2438_amd import build as B
    B.embed()
    lib = str(tmp_path / "libcwcssa_ubsan.so")
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")] + [
        f for f in B.HIP_FLAGS if f not in ("-O2",)] + [
        "-O1", "-g", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
        "-fno-sanitize-recover=all", "-shared-libsan",
        "-Wl,-rpath," + os.path.dirname(rt[-1]), "-shared", "-o", lib] + \
        [os.path.join(CSRC, s) for s in B.SOURCES] + ["-lhiprtc"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([sys.executable, "-c", HOST_EXERCISE, lib, ROOT], capture_output=True,
                       text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, (r.stdout[-1000:], r.stderr[-3000:])
    assert "ok" in r.stdout and "runtime error" not in r.stderr
