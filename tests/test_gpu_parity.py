"""GPU parity: the C-ABI library against the CPU oracle on identical seeded
inputs.  Integer results (counts, events, statuses, fired-leaf digests,
samples, moments) must match bit for bit, simulation times bit for bit,
mean/variance within 1e-12 relative."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_common import compare_stats, compare_trajectories, conservation_laws, gpu_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1010_2438_amd import Context
    c = Context(0)
    yield c
    c.close()


_models = {}


def model(ctx, m):
    from paper_1010_2438_amd import Model
    key = repr(m)
    if key not in _models:
        _models[key] = Model(ctx, m)
    return _models[key]


def check(ctx, m, run, modes=("plain", "persistent"), tuning=None, threads=8):
    orc = oracle.simulate(m, run, want_samples=True, threads=threads)
    mo = model(ctx, m)
    for mode in modes:
        print("case", m["name"], "mode", mode, "G", run["n_instances"] * run["replicas"], flush=True)
        g = gpu_run(ctx, mo, run, mode=mode, tuning=tuning)
        compare_trajectories(g, orc)
        compare_stats(g, orc)
    return orc


def test_config0_lotka_volterra_full(ctx):
    """Configuration 0 at its full size: 64 LV replicas to t = 5."""
    m, run = W.config(0)
    check(ctx, m, run)


@pytest.mark.parametrize("name", ["birth_death", "isomerisation", "dimerisation",
                                  "paper_example", "transport", "receptor_binding"])
def test_small_models(ctx, name):
    m = getattr(W, name)()
    run = W.make_run(seed=3, replicas=300, dt=0.25, n_samples=41)
    check(ctx, m, run)


@pytest.mark.parametrize("which", ["one_cell", "seven_children"])
def test_lane_layout_wide_trees(ctx, which):
    """Lane layout at its largest tree (64 leaves: one cell of the
    multi-compartment model, 24 cells) and a 7-child transport model, both
    forms, 300 replicas."""
    m = (W.multi_compartment(3, n_cells_=1) if which == "one_cell"
         else W.transport(n_children=7))
    run = W.make_run(seed=5, replicas=300, dt=0.25, n_samples=41)
    check(ctx, m, run)


def test_gene_regulation_ragged(ctx):
    """Configuration 1's model, 333 replicas (not a multiple of the block)."""
    m, run = W.config(1, replicas=333)
    run = dict(run, n_samples=41)          # t_end = 20
    check(ctx, m, run)


def test_sweep_rate_table(ctx):
    """Configuration 2's sweep: per-instance rate rows (first 24 instances,
    5 replicas each) in both execution forms."""
    m, _ = W.config(1)
    tab, _ = W.sweep_rate_table(m, 4096, 2)
    run = W.make_run(seed=0, n_instances=24, replicas=5, dt=0.5, n_samples=21,
                     rate_table=tab[:24])
    check(ctx, m, run)


def test_init_table(ctx):
    m = W.lotka_volterra(x0=100, y0=100, k=(1.0, 0.01, 1.0))
    init = np.array([[100, 100], [50, 20], [0, 30], [7, 0]], np.int32)
    run = W.make_run(seed=11, n_instances=4, replicas=17, dt=0.1, n_samples=31,
                     init_table=init)
    check(ctx, m, run)


def test_terminal_statuses(ctx):
    m, run = W.config(0, replicas=70)
    check(ctx, m, dict(run, max_events=20000))                 # EVENT_CAP
    check(ctx, m, dict(run, count_cap=1010))                   # OVERFLOW
    check(ctx, W.pure_decay(2.0, 5), W.make_run(replicas=65, dt=0.5, n_samples=30))  # ABSORBED


def test_degenerate_sizes(ctx):
    m = W.isomerisation()
    check(ctx, m, W.make_run(seed=1, replicas=1, dt=0.1, n_samples=1))     # one sample, one replica
    check(ctx, m, W.make_run(seed=2, replicas=64, dt=0.1, n_samples=2))
    z = W.isomerisation(a0=0, b0=0)                                          # empty: absorbed at t=0
    check(ctx, z, W.make_run(seed=2, replicas=10, dt=0.1, n_samples=5))


@pytest.mark.parametrize("tuning", [{"block_size": 64, "waves_per_simd": 1},
                                    {"block_size": 128, "waves_per_simd": 4},
                                    {"block_size": 256, "waves_per_simd": 8}])
def test_persistent_tuning_invariance(ctx, tuning):
    """Launch shape changes nothing: bit-identical to the oracle for any
    block shape and resident-wave count."""
    m, run = W.config(0, replicas=200)
    run = dict(run, n_samples=21)
    check(ctx, m, run, modes=("persistent",), tuning=tuning)


_refill_oracle = {}


def refill_case():
    """A sweep large enough that the persistent grid must refill (more
    trajectories than 65536 resident lanes at one wave per SIMD): 2800
    instances x 37 replicas of A <-> B with instance rates scaled over two
    decades, so trajectory lengths differ by about 100x."""
    m = W.isomerisation(k1=1.0, k2=3.0, a0=12, b0=0)
    tab, _ = W.sweep_rate_table(m, 2800, 5)
    run = W.make_run(seed=21, n_instances=2800, replicas=37, dt=0.2, n_samples=11,
                     rate_table=tab)
    if "o" not in _refill_oracle:
        _refill_oracle["o"] = oracle.simulate(m, run, want_samples=True, threads=8)
    return m, run, _refill_oracle["o"]


@pytest.mark.parametrize("chunk", [1, 64, 100])
def test_persistent_refill_chunks(ctx, chunk):
    """The persistent form's queue refill (lanes claiming single items, or
    wavefronts claiming chunks that cross instance boundaries) gives results
    bit-identical to the oracle's, trajectory by trajectory and in the
    per-instance moments."""
    m, run, orc = refill_case()
    print("case refill chunk", chunk, flush=True)
    g = gpu_run(ctx, model(ctx, m), run, mode="persistent",
                tuning={"block_size": 64, "waves_per_simd": 1, "refill_chunk": chunk})
    compare_trajectories(g, orc)
    compare_stats(g, orc)


@pytest.mark.parametrize("tuning", [{"sample_slots": 1, "refill_chunk": 64},
                                    {"sample_slots": 64, "refill_chunk": 256, "block_size": 128}])
def test_sampling_buffer_depth(ctx, tuning):
    """The accumulator rows kept per wavefront (1: every sample written back
    at once, up to 64) change nothing in the results."""
    m, run, orc = refill_case()
    print("case depth", tuning, flush=True)
    t = dict({"block_size": 64, "waves_per_simd": 1}, **tuning)
    g = gpu_run(ctx, model(ctx, m), run, mode="persistent", tuning=t)
    compare_trajectories(g, orc)
    compare_stats(g, orc)


@pytest.mark.parametrize("bad", [{"refill_chunk": 32}, {"sample_slots": 3},
                                 {"sample_slots": 128}])
def test_tuning_validation(ctx, bad):
    from paper_1010_2438_amd import CwcError
    m, run = W.config(0)
    with pytest.raises(CwcError) as e:
        gpu_run(ctx, model(ctx, m), run, mode="persistent",
                tuning=dict({"block_size": 64, "waves_per_simd": 1}, **bad))
    assert e.value.code == -1


# ---------------------------------------------------------------- pair layout

def bursts(sizes=(600, 900, 1500, 3000, 5000, 700), name="bursts"):
    """Six species made in bursts of 600 to 5000 molecules and lost one at a
    time, and a seventh only made, in bursts of 300.  The change table takes
    the byte layout: signed half-word fields for the six, an unsigned
    half-word for the seventh, four words per leaf."""
    rules = []
    for i, b in enumerate(sizes):
        rules.append(W._local(0, {}, {i: b}, 1.0))
        rules.append(W._local(0, {i: 1}, {}, 1.0))
    rules.append(W._local(0, {}, {6: 300}, 0.5))
    return W._single(name, [f"X{i}" for i in range(7)], rules, [0] * 7)


def bursts_dense():
    """bursts() with one burst of 40000: its 17-bit change field does not fit
    a half-word, so the table takes the dense layout (fields of their own
    widths in two words) and the cells that do not fit there take their
    change from per-digit 32-bit leaf masks."""
    return bursts(sizes=(600, 900, 1500, 3000, 40000, 700), name="bursts_dense")


def bursts_wide():
    """bursts() plus 26 isomerisations among four more species: 39 slots,
    a 64-leaf tree, so the table takes the dense layout and the cells whose
    change fields do not fit it take the 64-bit leaf-mask path."""
    m = bursts()
    rules = list(m["rules"])
    for k in range(26):
        a, c = 7 + (k % 4), 7 + ((k + 1) % 4)
        rules.append(W._local(0, {a: 1}, {c: 1}, 0.5 + 0.1 * k))
    return W._single("bursts_wide", ["X%d" % i for i in range(11)], rules,
                     [0] * 7 + [50, 50, 50, 50])


@pytest.mark.parametrize("table", ["bytes", "dense", "wide"])
@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_large_changes(ctx, lanes, table):
    """Large net changes per event, each change-table layout, one, two and
    four lanes per trajectory (the groups' per-lane tables, or every lane
    keeping every cell where a change does not fit a half-word) and both
    forms; with a cap below the largest burst the trajectories end in
    overflow with the state before the burst."""
    m = {"bytes": bursts, "dense": bursts_dense, "wide": bursts_wide}[table]()
    tuning = {2: PAIR, 4: QUAD}.get(lanes)
    run = W.make_run(seed=13, replicas=300, dt=0.1, n_samples=21)
    check(ctx, m, run, tuning=tuning)
    orc = check(ctx, m, dict(run, count_cap=4000), tuning=tuning)
    assert (orc["status"] == 2).sum() > 100


PAIR = {"lanes_per_replica": 2, "block_size": 64, "waves_per_simd": 1}


@pytest.mark.parametrize("name", ["birth_death", "isomerisation", "transport",
                                  "receptor_binding", "lotka_volterra"])
def test_pair_layout_small_models(ctx, name):
    """Two lanes per trajectory: bit-identical to the oracle in both forms."""
    m = getattr(W, name)()
    run = W.make_run(seed=7, replicas=300, dt=0.25, n_samples=41)
    check(ctx, m, run, tuning=PAIR)


def test_pair_layout_tables(ctx):
    """Two lanes per trajectory with per-instance rate rows and initial
    states."""
    m, _ = W.config(1)
    tab, _ = W.sweep_rate_table(m, 4096, 2)
    check(ctx, m, W.make_run(seed=0, n_instances=24, replicas=5, dt=0.5, n_samples=21,
                             rate_table=tab[:24]), tuning=PAIR)
    lv = W.lotka_volterra(x0=100, y0=100, k=(1.0, 0.01, 1.0))
    init = np.array([[100, 100], [50, 20], [0, 30], [7, 0]], np.int32)
    check(ctx, lv, W.make_run(seed=11, n_instances=4, replicas=17, dt=0.1, n_samples=31,
                              init_table=init), tuning=PAIR)


def test_pair_layout_needs_two_leaves(ctx):
    from paper_1010_2438_amd import CwcError
    with pytest.raises(CwcError) as e:
        gpu_run(ctx, model(ctx, W.dimerisation()), W.make_run(replicas=8, n_samples=3),
                tuning=PAIR)
    assert e.value.code == -2


def test_pair_layout_gene_regulation_and_wide_tree(ctx):
    m, run = W.config(1, replicas=333)
    check(ctx, m, dict(run, n_samples=41), tuning=PAIR)
    check(ctx, W.multi_compartment(3, n_cells_=1),
          W.make_run(seed=5, replicas=300, dt=0.25, n_samples=41), tuning=PAIR)


def test_pair_layout_statuses(ctx):
    m, run = W.config(0, replicas=70)
    check(ctx, m, dict(run, max_events=20000), tuning=PAIR)
    check(ctx, m, dict(run, count_cap=1010), tuning=PAIR)
    # absorbing: two species that only decay
    decay2 = W._single("decay2", ["A", "B"], [W._local(0, {0: 1}, {}, 2.0),
                                              W._local(0, {1: 1}, {}, 1.0)], [5, 3])
    check(ctx, decay2, W.make_run(replicas=65, dt=0.5, n_samples=30), tuning=PAIR)


@pytest.mark.parametrize("chunk", [1, 64])
def test_pair_layout_refill(ctx, chunk):
    """Pairs claiming queue items (more trajectories than resident pairs)."""
    m, run, orc = refill_case()
    g = gpu_run(ctx, model(ctx, m), run, mode="persistent",
                tuning=dict(PAIR, refill_chunk=chunk))
    compare_trajectories(g, orc)
    compare_stats(g, orc)



QUAD = {"lanes_per_replica": 4, "block_size": 64, "waves_per_simd": 1}


@pytest.mark.parametrize("name", ["transport", "receptor_binding", "lotka_volterra",
                                  "transport7"])
def test_quad_layout_small_models(ctx, name):
    """Four lanes per trajectory: bit-identical to the oracle in both forms."""
    m = W.transport(n_children=7) if name == "transport7" else getattr(W, name)()
    run = W.make_run(seed=17, replicas=300, dt=0.25, n_samples=41)
    check(ctx, m, run, tuning=QUAD)


def test_quad_layout_gene_regulation_tables_and_wide_tree(ctx):
    """Four lanes per trajectory on configuration 1's model (ragged 333
    replicas), with per-instance rate rows, and on a 64-leaf tree."""
    m, run = W.config(1, replicas=333)
    check(ctx, m, dict(run, n_samples=41), tuning=QUAD)
    tab, _ = W.sweep_rate_table(m, 4096, 2)
    check(ctx, m, W.make_run(seed=0, n_instances=24, replicas=5, dt=0.5, n_samples=21,
                             rate_table=tab[:24]), tuning=QUAD)
    check(ctx, W.multi_compartment(3, n_cells_=1),
          W.make_run(seed=5, replicas=300, dt=0.25, n_samples=41), tuning=QUAD)


def test_quad_layout_statuses_and_large_changes(ctx):
    m, run = W.config(0, replicas=70)
    check(ctx, m, dict(run, max_events=20000), tuning=QUAD)
    check(ctx, m, dict(run, count_cap=1010), tuning=QUAD)
    lv = W.lotka_volterra(x0=100, y0=100, k=(1.0, 0.01, 1.0))
    init = np.array([[100, 100], [50, 20], [0, 30], [7, 0]], np.int32)
    check(ctx, lv, W.make_run(seed=11, n_instances=4, replicas=17, dt=0.1, n_samples=31,
                              init_table=init), tuning=QUAD)
    bm = bursts()
    brun = W.make_run(seed=13, replicas=300, dt=0.1, n_samples=21)
    check(ctx, bm, brun, tuning=QUAD)
    check(ctx, bm, dict(brun, count_cap=4000), tuning=QUAD)


_refill4_oracle = {}


def refill_case4():
    """refill_case's sweep on a four-leaf model (A <-> B, A -> 0, 0 -> A)."""
    m = W._single("iso4", ["A", "B"], [W._local(0, {0: 1}, {1: 1}, 1.0),
                                       W._local(0, {1: 1}, {0: 1}, 3.0),
                                       W._local(0, {0: 1}, {}, 0.2),
                                       W._local(0, {}, {0: 1}, 2.0)], [12, 0])
    tab, _ = W.sweep_rate_table(m, 2800, 5)
    run = W.make_run(seed=23, n_instances=2800, replicas=37, dt=0.2, n_samples=11,
                     rate_table=tab)
    if "o" not in _refill4_oracle:
        _refill4_oracle["o"] = oracle.simulate(m, run, want_samples=True, threads=8)
    return m, run, _refill4_oracle["o"]


@pytest.mark.parametrize("chunk", [1, 64])
def test_quad_layout_refill(ctx, chunk):
    """Quads claiming queue items (103,600 trajectories, more than the
    resident quads)."""
    m, run, orc = refill_case4()
    g = gpu_run(ctx, model(ctx, m), run, mode="persistent",
                tuning=dict(QUAD, refill_chunk=chunk))
    compare_trajectories(g, orc)
    compare_stats(g, orc)


def test_quad_layout_needs_four_leaves(ctx):
    from paper_1010_2438_amd import CwcError
    decay2 = W._single("decay2", ["A", "B"], [W._local(0, {0: 1}, {}, 2.0),
                                              W._local(0, {1: 1}, {}, 1.0)], [5, 3])
    with pytest.raises(CwcError) as e:
        gpu_run(ctx, model(ctx, decay2), W.make_run(replicas=8, n_samples=3), tuning=QUAD)
    assert e.value.code == -2


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_persistent_grid_holding_every_item(ctx, lanes):
    """A persistent grid that holds every trajectory (16 requested waves per
    SIMD) runs the queue-free kernel with the instances still taken
    longest-first: results are the oracle's, trajectory by trajectory."""
    from paper_1010_2438_amd import Run
    m, run, orc = refill_case4() if lanes == 4 else refill_case()
    tun = {"block_size": 256, "waves_per_simd": 16, "lanes_per_replica": lanes}
    r = Run(ctx, model(ctx, m), run, mode="persistent", tuning=tun)
    fam = {1: "cwc_lane", 2: "cwc_pair", 4: "cwc_quad"}[lanes]
    assert r.kernel_name() == fam + "_plain_table"
    r.close()
    g = gpu_run(ctx, model(ctx, m), run, mode="persistent", tuning=tun)
    compare_trajectories(g, orc)
    compare_stats(g, orc)


def test_kernel_names(ctx):
    """cwc_run_kernel_name names the dispatched simulation kernel."""
    from paper_1010_2438_amd import Run
    m, run, _ = refill_case()
    mo = model(ctx, m)
    lv = model(ctx, W.lotka_volterra())
    lv_run = W.make_run(replicas=64, n_samples=3)
    cases = [(mo, run, "plain", {"lanes_per_replica": 1}, "cwc_lane_plain_table"),
             (mo, run, "persistent", {"lanes_per_replica": 2, "block_size": 64,
                                      "waves_per_simd": 1}, "cwc_pair_persistent_table"),
             (lv, lv_run, "plain", {"lanes_per_replica": 4}, "cwc_quad_plain_shared"),
             (lv, lv_run, "persistent", {"lanes_per_replica": 64}, "cwc_wave_plain_shared")]
    for mobj, rr, mode, tun, name in cases:
        r = Run(ctx, mobj, rr, mode=mode, tuning=tun)
        assert r.kernel_name() == name
        r.wait()
        r.close()

# ---------------------------------------------------------------- wave layout

def test_config3_multicompartment(ctx):
    """Configuration 3's model (32 cells in an outer compartment, 396
    cells, 836 slots): wavefront-per-replica layout, 24 replicas to t = 10."""
    m, run = W.config(3, replicas=24)
    run = dict(run, n_samples=21)
    mo = model(ctx, m)
    assert mo.info["layout"] == 1
    check(ctx, m, run)


@pytest.mark.parametrize("name", ["birth_death", "lotka_volterra", "paper_example",
                                  "transport", "receptor_binding", "gene_regulation"])
def test_small_models_wave_layout(ctx, name):
    """The same models forced into the wavefront layout match the oracle
    (and therefore the lane layout) bit for bit."""
    m = getattr(W, name)()
    run = W.make_run(seed=5, replicas=40, dt=0.25, n_samples=21)
    check(ctx, m, run, tuning={"lanes_per_replica": 64})


def test_wave_layout_largest_model(ctx):
    """The wavefront layout at its largest model: 64 compartments (63 cells
    in an outer one), one per lane, 768 count cells, 2048 leaves; both
    forms against the oracle."""
    m = W.multi_compartment(3, n_cells_=63)
    mo = model(ctx, m)
    assert mo.info["layout"] == 1 and mo.info["n_cells"] == 768
    check(ctx, m, W.make_run(seed=23, replicas=12, dt=0.2, n_samples=6))


def test_wave_layout_statuses(ctx):
    m = W.multi_compartment(3, n_cells_=5)
    run = W.make_run(seed=9, replicas=20, dt=0.5, n_samples=11)
    check(ctx, m, dict(run, max_events=700), tuning={"lanes_per_replica": 64})
    cap = max(max(r) for r in m["init"]) + 2          # first overflow comes quickly
    check(ctx, m, dict(run, count_cap=cap), tuning={"lanes_per_replica": 64})
    check(ctx, W.pure_decay(3.0, 4), W.make_run(replicas=9, dt=0.5, n_samples=12),
          tuning={"lanes_per_replica": 64})


def test_golden_term_without_rules(ctx):
    """The Sec. 2.1 term (tests/golden fixture) as a model with no rules:
    every trajectory is absorbed at t = 0 and every sample holds the term's
    count cells, with one lane, two lanes or a wavefront per trajectory."""
    from tests.test_oracle_golden import multiset, read_fixture
    fx = read_fixture("term_example_sec2_1.txt")
    sp = fx["species"].split()
    m = {"name": "term_example", "species": sp,
         "types": [{"name": "top", "wrap": False}, {"name": fx["comp_type"], "wrap": True}],
         "compartments": [{"type": 0, "parent": -1}, {"type": 1, "parent": 0}],
         "init": [multiset(sp, fx["top_content"]), multiset(sp, fx["comp_content"])],
         "init_wrap": [None, multiset(sp, fx["comp_wrap"])], "rules": []}
    want = np.array([int(x) for x in fx["cells"].split()], np.int32)
    run = W.make_run(seed=4, replicas=70, dt=0.5, n_samples=6)
    for lanes in (1, 2, 64):
        orc = check(ctx, m, run, tuning={"lanes_per_replica": lanes})
    assert (orc["samples"] == want).all()
    assert (orc["events"] == 0).all() and (orc["t_final"] == 0.0).all()
    assert (orc["status"] == 1).all()
