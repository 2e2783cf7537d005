"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
function include/cwcssa.h declares, validates model descriptors with the
documented error codes, and its generated device code compiles for gfx950."""
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cwcssa.h")


@pytest.fixture(scope="module")
def P():
    import paper_1010_2438_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1010_2438_amd import build
        build.build()
    P.load()
    return P


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cwc_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(P):
    L = P.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(P.SYMBOLS)
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True).stdout
    for n in names:
        assert re.search(r"\sT\s%s$" % n, out, re.M), n
    assert L.cwc_abi_version() == 2


def test_context_without_device_fails_cleanly(P):
    import ctypes
    h = ctypes.c_void_p()
    rc = P.load().cwc_ctx_create(0, None, 0, ctypes.byref(h))
    # no GPU in this container: a clean CWC_E_DEVICE, never a crash
    import torch
    if not torch.cuda.is_available():
        assert rc == -4 and b"device" in P.load().cwc_last_error()


def code(P, model):
    try:
        P.cwc_codegen(model)
        return 0
    except P.CwcError as e:
        return e.code


def test_validation_errors(P):
    good = W.lotka_volterra()
    assert code(P, good) == 0
    bad = W.lotka_volterra()
    bad["rules"][0]["k"] = 0.0
    assert code(P, bad) == -1                                   # k <= 0
    bad = W.lotka_volterra()
    bad["rules"][0]["k"] = float("nan")
    assert code(P, bad) == -1
    bad = W.lotka_volterra()
    bad["rules"][1]["lhs"]["p"] = {0: 2, 1: 1}                  # order 3
    assert code(P, bad) == -2
    bad = W.lotka_volterra()
    bad["rules"][0]["lhs"]["p"] = {5: 1}                        # species out of range
    assert code(P, bad) == -1
    bad = W.lotka_volterra()
    bad["init"] = [[-1, 3]]
    assert code(P, bad) == -1
    bad = W.transport()
    bad["compartments"][1]["parent"] = 2                        # not preorder
    assert code(P, bad) == -1
    bad = W.transport()
    bad["rules"][0]["lhs"] = {"w": {0: 1}}                      # wrap on a label without one
    assert code(P, bad) == -1
    bad = W.lotka_volterra()
    bad["rules"][0]["lhs"] = {"c": {0: 1}}                      # child region in a local rule
    assert code(P, bad) == -1
    big = W.multi_compartment(3, n_cells_=70)                   # > 64 compartments, > 64 leaves
    assert code(P, big) == -2


def test_layout_choice(P):
    for m, lay in ((W.lotka_volterra(), "lane"), (W.gene_regulation(), "lane"),
                   (W.multi_compartment(), "wavefront")):
        assert ("(%s-per-replica layout)" % lay) in P.cwc_codegen(m)


@pytest.mark.parametrize("which", [0, 3])
def test_generated_code_compiles(P, which, tmp_path):
    """The device code generated for the benchmark models compiles offline
    for gfx950 with the library's flags and needs no scratch memory."""
    src = P.cwc_codegen(W.config(which)[0])
    f = tmp_path / "m.hip"
    f.write_text(src)
    r = subprocess.run(
        ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "--offload-device-only",
         "-c", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", "-include", "hip/hip_runtime.h", str(f), "-o",
         str(tmp_path / "m.o"), "-Rpass-analysis=kernel-resource-usage"],
        capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    assert scratch and max(scratch) == 0


def test_algorithmic_work_accounting(P):
    """The roofline's work unit for the LV model, by hand: P = 4 leaves
    (depth 2) -> 195 + 1 + 5*2 = 206 fixed (Philox 10 rounds x (2 wide
    multiplies at 4 slots + 4 xor) = 120; its key adds act on the run seed,
    the same in every lane, so they are scalar work); per fired slot: update 2 per
    changed cell, re-evaluation of dependent slots (order 1: 2, A+B: 4) and
    the distinct tree nodes above them:
      X->2X : 2 + (2 + 4) + |{2,1}|   = 10
      X+Y   : 4 + (2 + 4 + 2) + |{2,3,1}| = 15
      Y->0  : 2 + (4 + 2) + |{2,3,1}| = 11      mean 12 -> 218."""
    info = P.cwc_model_describe(W.lotka_volterra())
    assert info["n_leaves"] == 4 and info["n_slots"] == 3
    assert info["alg_slots_per_event"] == 218.0
    g = P.cwc_model_describe(W.gene_regulation())
    assert (g["n_cells"], g["n_slots"], g["n_leaves"], g["p_local"]) == (20, 20, 32, 16)
    c3 = P.cwc_model_describe(W.multi_compartment())
    assert (c3["n_cells"], c3["n_slots"], c3["n_leaves"], c3["layout"]) == (396, 836, 2048, 1)


def test_confidence_bands(P):
    """cwc_stats_confidence against scipy's Student-t distribution (an
    independent implementation): the returned quantile puts exactly the
    requested tail beyond it (scipy's sf, 1e-12 relative) and agrees with
    scipy's ppf to that routine's own accuracy; 50/90/99/99.9999 % bands,
    n from 2 to 10^6; NaN below two trajectories."""
    from scipy import stats
    rng = np.random.default_rng(3)
    n = np.array([0, 1, 2, 3, 5, 10, 21, 40, 41, 64, 1000, 16384, 1000000], np.int64)
    var = rng.uniform(0.5, 50.0, size=(len(n), 4))
    for level in (0.5, 0.9, 0.99, 0.999999):
        w = P.confidence(var, n, level)
        assert np.isnan(w[:2]).all()
        t = w[2:] / np.sqrt(var[2:] / n[2:, None])
        q = 0.5 - level / 2
        assert np.allclose(stats.t.sf(t, (n[2:] - 1)[:, None]), q, rtol=1e-12, atol=0)
        ref = stats.t.ppf(0.5 + level / 2, n[2:] - 1)
        assert np.allclose(t, ref[:, None], rtol=5e-10, atol=0)   # scipy ppf: ~1e-10
    with pytest.raises(P.CwcError):
        P.confidence(var, n, 1.5)


def test_bench_refuses_several_gpus():
    """This simulator runs on one GPU: the benchmark says so and exits 2
    before touching a device."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr
