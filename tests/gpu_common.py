"""Helpers shared by the GPU tests: run a model through the C-ABI library and
through the oracle on the same seeded inputs, and compare element by element."""
import math

import numpy as np

import oracle

RESULT_KEYS = ("events", "status", "digest", "n_recorded", "final_counts")


def gpu_run(ctx, model_obj, run, mode="plain", want_traj=True, want_digest=True,
            tuning=None):
    from paper_1010_2438_amd import Run
    r = Run(ctx, model_obj, run, mode=mode, want_traj=want_traj,
            want_digest=want_digest, tuning=tuning)
    r.wait()
    out = r.counters()
    out["mean"], out["var"], out["n"] = r.stats()
    out["s1"], out["s2_hi32"], out["s2_lo32"], _ = r.moments()
    if want_traj:
        out["samples"] = per_trajectory(r.trajectories())
    r.close()
    return out


def per_trajectory(t):
    """The library's sample layout [sample][cell][trajectory] as
    [trajectory][sample][cell] (the oracle's), copied in blocks of
    trajectories so each read is a run of contiguous words."""
    K1, C, G = t.shape
    out = np.empty((G, K1, C), t.dtype)
    step = 8192
    for g0 in range(0, G, step):
        out[g0:g0 + step] = t[:, :, g0:g0 + step].transpose(2, 0, 1)
    return out


def same_float(a, b):
    """Bitwise equality of float arrays, NaN == NaN."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


def compare_trajectories(gpu, orc, g_index=None, check_samples=True):
    """Per-trajectory results equal bit for bit.  g_index: rows of the GPU
    arrays that correspond to the oracle's rows (default: all)."""
    sel = slice(None) if g_index is None else g_index
    for key in RESULT_KEYS:
        a = np.asarray(gpu[key])[sel]
        b = np.asarray(orc[key])
        assert np.array_equal(a, b), "%s differs at %s" % (
            key, np.argwhere(a != b)[:5].tolist())
    assert same_float(np.asarray(gpu["t_final"])[sel], orc["t_final"]), "t_final differs"
    if check_samples and "samples" in orc and "samples" in gpu:
        gs = np.asarray(gpu["samples"])[sel]
        for i, nr in enumerate(orc["n_recorded"]):
            assert np.array_equal(gs[i, :nr], orc["samples"][i, :nr]), "samples differ row %d" % i


def compare_stats(gpu, orc):
    """Exact integer moments equal; mean and variance within 1e-12 relative
    (both NaN where fewer than 1 / 2 trajectories contributed)."""
    assert np.array_equal(gpu["n"], orc["n"].astype(np.int64))
    assert np.array_equal(gpu["s1"], orc["s1"])
    s2_gpu = [int(h) * 2 ** 32 + int(l) for h, l in
              zip(gpu["s2_hi32"].ravel(), gpu["s2_lo32"].ravel())]
    s2_orc = [int(h) * 2 ** 64 + int(l) for h, l in
              zip(orc["s2_hi"].ravel(), orc["s2_lo"].ravel())]
    assert s2_gpu == s2_orc
    for key in ("mean", "var"):
        a, b = gpu[key], orc[key]
        both_nan = np.isnan(a) & np.isnan(b)
        ok = both_nan | (a == b)
        if not ok.all():
            rel = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
            rel[both_nan] = 0
            assert np.nanmax(rel) <= 1e-12, (key, np.nanmax(rel))


def integer_null_space(rows, C):
    """Integer basis of the vectors w with r . w = 0 for every row r (exact
    rational elimination), as an int64 matrix [C][basis size]."""
    from fractions import Fraction
    from math import lcm
    rows = [[Fraction(x) for x in r] for r in rows]
    piv, r = [], 0
    for c in range(C):
        p = next((i for i in range(r, len(rows)) if rows[i][c] != 0), None)
        if p is None:
            continue
        rows[r], rows[p] = rows[p], rows[r]
        rows[r] = [x / rows[r][c] for x in rows[r]]
        for i in range(len(rows)):
            if i != r and rows[i][c] != 0:
                fct = rows[i][c]
                rows[i] = [a - fct * b for a, b in zip(rows[i], rows[r])]
        piv.append(c)
        r += 1
    basis = []
    for fc in (c for c in range(C) if c not in piv):
        w = [Fraction(0)] * C
        w[fc] = Fraction(1)
        for i, pc in enumerate(piv):
            w[pc] = -rows[i][fc]
        den = lcm(*[x.denominator for x in w])
        basis.append([int(x * den) for x in w])
    return np.array(basis, dtype=np.int64).T.reshape(C, len(basis))


def conservation_laws(model):
    """Integer basis of the vectors w with w . delta = 0 for the net change
    delta of every slot of the oracle's flattening: w . counts is the same
    in every state a trajectory reaches.  Int64 matrix [cells][laws]."""
    import oracle
    f = oracle.FlatModel(model)
    rows = []
    for leaf in range(f.n_leaves):
        if f.leaf_rule[leaf] < 0:
            continue
        v = [0] * f.n_cells
        for k in range(int(f.leaf_ndelta[leaf])):
            cell, d = (int(x) for x in f.leaf_delta[leaf, k])
            v[cell] += d
        rows.append(v)
    return integer_null_space(rows, f.n_cells)


def oracle_ids(model, run, ids, threads=16, want_samples=True):
    """The oracle's per-trajectory results for trajectories `ids` (any
    order, any spread over the id range), one oracle call per trajectory on
    `threads` host threads; rows in the order of `ids`."""
    import threading
    fm = oracle.FlatModel(model)
    ids = [int(i) for i in ids]
    rows = [None] * len(ids)

    def work(k):
        for q in range(k, len(ids), threads):
            rows[q] = oracle.simulate(model, run, g0=ids[q], g1=ids[q] + 1,
                                      want_samples=want_samples, want_stats=False, flat=fm)

    ts = [threading.Thread(target=work, args=(k,)) for k in range(max(1, min(threads, len(ids))))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    keys = RESULT_KEYS + ("t_final",) + (("samples",) if want_samples else ())
    return {k: np.concatenate([r[k] for r in rows]) for k in keys}
