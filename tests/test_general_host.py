"""Host: general CWC models (compartments created, dissolved and deleted at
run time) -- the generated device code of each workload model compiles for
gfx950 without scratch memory, and model validation rejects what the
engine does not do, without a device."""
import os
import subprocess
import tempfile

import pytest

import workloads as W

MODELS = [W.cell_birth_death(), W.cell_dissolution(), W.nested_export(),
          W.receptor_internalisation(), W.cell_colony(),
          W.general_from_fixed(W.multi_compartment(3))]


@pytest.fixture(scope="module")
def P():
    import paper_1010_2438_amd as P
    P.load()
    return P


@pytest.mark.parametrize("m", MODELS, ids=[m["name"] for m in MODELS])
def test_generated_code_compiles(P, m):
    src = P.gcodegen(m)
    assert "cwc_gen_persistent_table" in src
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "g.hip")
        open(path, "w").write(src)
        r = subprocess.run(
            [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-x", "hip", "--offload-arch=gfx950",
             "--offload-device-only", "-c", "-O3", "-std=c++17", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-include", "hip/hip_runtime.h", "-Rpass-analysis=kernel-resource-usage",
             path, "-o", path + ".o"], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        assert "ScratchSize [bytes/lane]: 0" in r.stderr
        assert "ScratchSize [bytes/lane]: 1" not in r.stderr


def bad(m, **change):
    m = dict(m)
    m.update(change)
    return m


def test_validation(P):
    base = W.cell_dissolution()
    r0 = dict(base["rules"][0])
    cases = [
        bad(base, max_comp=65),                                             # > one wavefront
        bad(base, rules=[dict(r0, lhs={"c2": {0: 1}})]),                    # region beyond depth
        bad(base, rules=[dict(r0, lhs={"c": {0: 2, 1: 1}})]),               # order 3
        bad(base, rules=[dict(r0, k=0.0)]),                                 # k <= 0
        bad(base, rules=[dict(r0, action="delete", level=2)]),              # deletes what it lacks
        bad(base, term=[base["term"][1], base["term"][0]]),                 # not preorder
        bad(base, term=base["term"] + [dict(base["term"][0], parent=0, label=9)]),  # label
    ]
    for m in cases:
        with pytest.raises(P.CwcError):
            P.gcodegen(m)
