"""Batched execution: every member of a batch ends in exactly the state it reaches alone.

Members mix 2D/3D lattices and random regular graphs of degree 3..6, one to five words
per site, different m, densities, seeds and sweep counts (so they finish at different
steps).  The reference for each member is the same sim advanced alone with ka_sweep (itself
parity-tested against the oracle); a few members are also checked against the oracle
directly.  Launch shapes (workgroup size, persistent grid, graph capture, autotuning) must
not change any bit, and members added while the batch runs must also match.
"""
import numpy as np
import pytest

from paper_1710_05155_amd import ka

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


MEMBERS = [
    # kind, size, z, m, rho, R, seed, sweeps
    ("lat", (2, 8), 4, 2, 0.6, 64, 1, 5),
    ("lat", (2, 12), 4, 1, 0.5, 128, 2, 9),
    ("lat", (2, 64), 4, 2, 0.7, 64, 3, 4),
    ("lat", (3, 8), 6, 3, 0.8, 256, 4, 3),
    ("lat", (3, 12), 6, 2, 0.65, 64, 5, 6),
    ("lat", (2, 32), 4, 3, 0.85, 192, 6, 2),
    ("rrg", 64, 3, 1, 0.5, 64, 7, 7),
    ("rrg", 300, 6, 3, 0.8, 128, 8, 3),
    ("rrg", 2000, 4, 2, 0.65, 64, 9, 5),
    ("rrg", 500, 5, 3, 0.7, 192, 10, 4),
    ("rrg", 1000, 3, 0, 0.55, 320, 11, 2),
    ("lat", (3, 16), 6, 3, 0.88, 128, 12, 1),
]


def _graph(spec):
    kind, size, z = spec[0], spec[1], spec[2]
    if kind == "lat":
        return ka.ka_graph_lattice(*size)
    return ka.ka_graph_rrg(size, z, 31 + size)


def _make(spec, g, stream=None):
    _, _, _, m, rho, R, seed, _ = spec
    return ka.ka_init(g, m, rho, seed, R, stream=stream)


def _solo_states(graphs):
    out = []
    for spec, g in zip(MEMBERS, graphs):
        s = _make(spec, g)
        ka.ka_sweep(s, spec[7])
        out.append(ka.ka_get_state(s))
        s.free()
    return out


def _run_batch(graphs, options=()):
    b = ka.ka_batch_create(64)
    for opt, val in options:
        ka.ka_batch_set_option(b, opt, val)
    sims = []
    for spec, g in zip(MEMBERS, graphs):
        s = _make(spec, g)
        ka.ka_batch_add(b, s, spec[7])
        sims.append(s)
    ka.ka_batch_wait_all(b)
    states = [ka.ka_get_state(s) for s in sims]
    info = ka.ka_batch_info(b)
    b.free()
    return states, info


@pytest.fixture(scope="module")
def graphs():
    return [_graph(spec) for spec in MEMBERS]


@pytest.fixture(scope="module")
def solo(graphs):
    _say("batch: solo references")
    return _solo_states(graphs)


def _assert_same(states, solo):
    for k, (a, b) in enumerate(zip(states, solo)):
        for x, y in zip(a, b):
            assert np.array_equal(np.asarray(x), np.asarray(y)), f"member {k} ({MEMBERS[k][:2]})"


@pytest.mark.parametrize("options", [
    (),                                                                         # autotuned, graphs
    ((ka.KA_BOPT_BLOCK, 128), (ka.KA_BOPT_GRAPH_STEPS, 0)),
    ((ka.KA_BOPT_BLOCK, 512), (ka.KA_BOPT_GRAPH_STEPS, 5)),
    ((ka.KA_BOPT_BLOCK, 256), (ka.KA_BOPT_GRAPH_STEPS, 64)),
])
def test_batch_members_equal_solo(graphs, solo, options):
    _say(f"batch options {options}")
    states, info = _run_batch(graphs, options)
    _assert_same(states, solo)
    assert info[1] == 0  # all members detached


def test_block_changes_between_queued_runs(graphs, solo):
    """The workgroup size changes between ka_batch_run calls while earlier steps (and the
    member-table uploads enqueued with them) are still pending on the stream: each upload
    must carry the table of its own segment, so every member still ends in its solo state."""
    _say("batch: block changes with queued work")
    b = ka.ka_batch_create(64)
    ka.ka_batch_set_option(b, ka.KA_BOPT_GRAPH_STEPS, 2)
    sims = []
    for spec, g in zip(MEMBERS, graphs):
        s = _make(spec, g)
        ka.ka_batch_add(b, s, spec[7])
        sims.append(s)
    blocks = [128, 512, 256, 512, 128, 256]
    q = 0
    while ka.ka_batch_steps_left(b) > 0:
        ka.ka_batch_set_option(b, ka.KA_BOPT_BLOCK, blocks[q % len(blocks)])
        ka.ka_batch_run(b, 3)
        q += 1
    ka.ka_batch_wait_all(b)
    states = [ka.ka_get_state(s) for s in sims]
    b.free()
    _assert_same(states, solo)
    for s in sims:
        s.free()


def test_batch_members_match_oracle(oracle):
    """Two members checked against the oracle directly (all replicas, state and counts)."""
    g2 = ka.ka_graph_lattice(2, 12)
    og2 = oracle.lattice(2, 12)
    gr = ka.ka_graph_rrg(300, 4, 5)
    ogr = oracle.graph_from_adjacency(oracle.rrg_adjacency(300, 4, 5)[0])
    _say("batch vs oracle")
    b = ka.ka_batch_create(4)
    a = ka.ka_init(g2, 2, 0.6, 21, 128)
    c = ka.ka_init(gr, 1, 0.55, 22, 64)
    ka.ka_batch_add(b, a, 6)
    ka.ka_batch_add(b, c, 9)
    ka.ka_batch_wait_all(b)
    for sim, og, m, rho, seed, R, n in [(a, og2, 2, 0.6, 21, 128, 6), (c, ogr, 1, 0.55, 22, 64, 9)]:
        orc = oracle.Sim(og, m, oracle.k_from_rho(og.N, rho), seed, range(R))
        orc.sweep(n)
        n_, n0_, f_, t_ = ka.ka_get_state(sim)
        assert t_ == n
        assert np.array_equal(n_, oracle.pack(orc.occ)) and np.array_equal(f_, oracle.pack(orc.moved))
        t, dens, ov, pers = ka.ka_observe(sim)
        od, oo, op = orc.observe()
        assert np.array_equal(dens, od) and np.array_equal(ov, oo) and np.array_equal(pers, op)


@pytest.mark.parametrize("solo_bytes", [None, 1 << 16])
def test_members_added_while_running(graphs, solo, solo_bytes):
    """Continuous batching: members join after the batch has started and leave as they
    finish; each still ends in its solo state (also with some members run one at a time,
    solo members queueing behind each other as they join)."""
    _say(f"batch: staggered admission, solo bytes {solo_bytes}")
    b = ka.ka_batch_create(8)  # fewer slots than members: slots are reused
    ka.ka_batch_set_option(b, ka.KA_BOPT_GRAPH_STEPS, 4)
    if solo_bytes is not None:
        ka.ka_batch_set_option(b, ka.KA_BOPT_SOLO_BYTES, solo_bytes)
    pending = list(range(len(MEMBERS)))
    sims = {}
    results = {}
    rounds = 0
    while pending or b.members:
        while pending and len(b.members) < 8:
            k = pending.pop(0)
            s = _make(MEMBERS[k], graphs[k])
            slot = ka.ka_batch_add(b, s, MEMBERS[k][7])
            sims[slot] = (k, s)
        ka.ka_batch_run(b, 3)
        for slot in ka.ka_batch_poll(b):
            k, s = sims.pop(slot)
            results[k] = ka.ka_get_state(s)
            s.free()
        rounds += 1
        assert rounds < 10_000
        if not pending and b.members and ka.ka_batch_steps_left(b) == 0:
            ka.ka_batch_wait_all(b)
            for slot, (k, s) in list(sims.items()):
                results[k] = ka.ka_get_state(s)
            sims.clear()
    b.free()
    assert sorted(results) == list(range(len(MEMBERS)))
    _assert_same([results[k] for k in range(len(MEMBERS))], solo)


def test_batch_errors(graphs):
    b = ka.ka_batch_create(1)
    s = _make(MEMBERS[0], graphs[0])
    ka.ka_batch_add(b, s, 2)
    with pytest.raises(ka.KaError) as e:
        ka.ka_sweep(s, 1)
    assert e.value.code == ka.KA_ESTATE
    s2 = _make(MEMBERS[1], graphs[1])
    with pytest.raises(ka.KaError) as e:
        ka.ka_batch_add(b, s2, 1)          # full
    assert e.value.code == ka.KA_ESTATE
    b2 = ka.ka_batch_create(2)
    with pytest.raises(ka.KaError):
        ka.ka_batch_add(b2, s, 1)          # already a member elsewhere
    ka.ka_batch_wait_all(b)
    assert s.t == 2
    ka.ka_sweep(s, 1)                      # detached: usable again
    b.free()
    b2.free()


def test_batch_shared_noise_members_equal_solo(graphs):
    """Members with shared noise (KA_OPT_NOISE = 1) next to members with independent noise
    end bit-identical to their solo runs with the same setting."""
    _say("batch: mixed noise settings")
    shared = [k % 2 == 0 for k in range(len(MEMBERS))]
    ref = []
    for spec, g, sh in zip(MEMBERS, graphs, shared):
        s = _make(spec, g)
        ka.ka_set_option(s, ka.KA_OPT_NOISE, int(sh))
        ka.ka_sweep(s, spec[7])
        ref.append(ka.ka_get_state(s))
        s.free()
    b = ka.ka_batch_create(64)
    sims = []
    for spec, g, sh in zip(MEMBERS, graphs, shared):
        s = _make(spec, g)
        ka.ka_set_option(s, ka.KA_OPT_NOISE, int(sh))
        ka.ka_batch_add(b, s, spec[7])
        sims.append(s)
    ka.ka_batch_wait_all(b)
    states = [ka.ka_get_state(s) for s in sims]
    b.free()
    _assert_same(states, ref)


BUDGET_MEMBERS = [
    # large (working set 64 KiB: 2D L=64, 64 replicas, C=8) and small members
    ("lat", (2, 64), 4, 2, 0.7, 64, 40, 5),
    ("lat", (2, 64), 4, 1, 0.6, 64, 41, 5),
    ("rrg", 2000, 4, 2, 0.65, 64, 42, 3),
    ("lat", (2, 64), 4, 3, 0.8, 64, 43, 5),
    ("lat", (2, 8), 4, 2, 0.6, 64, 44, 7),
    ("lat", (2, 64), 4, 2, 0.5, 64, 45, 5),
]


# Steps under each budget, worked out by hand from the admission rule: large members are
# the 2D L=64 ones (64 KiB, 40 steps) and, below 250 KiB, the graph (31.25 KiB, 15 classes x
# 3 sweeps = 45 steps); the small 2D L=8 member takes 56 steps from the start.
#   128 KiB: two L=64 to step 40, then graph + L=64 (to 85 / 80), then the last L=64 from 80 to 120.
#   192 KiB: two L=64 + graph at once; at 40 the other two L=64 start, to 80.
#    64 KiB: one large member at a time: 40, 80, 125 (graph), 165, 205.
#     1 MiB: nothing is large; the small member's 56 steps set the length.
@pytest.mark.parametrize("budget,expected_steps", [(1 << 17, 120), (3 << 16, 80), (1 << 16, 205), (1 << 20, 56)])
def test_cache_budget_members_equal_solo(budget, expected_steps):
    """Infinity-Cache-aware admission (KA_BOPT_CACHE_BUDGET): members whose working set is
    at least 1/8 of the budget start only while they fit it next to the large members still
    running, in the order added.  ka_batch_steps_left projects those admissions exactly, so
    running that many steps completes every member, and each ends in its solo state."""
    import time
    _say(f"batch: cache budget {budget}")
    graphs = [_graph(spec) for spec in BUDGET_MEMBERS]
    solo = []
    for spec, g in zip(BUDGET_MEMBERS, graphs):
        s = _make(spec, g)
        ka.ka_sweep(s, spec[7])
        solo.append(ka.ka_get_state(s))
        s.free()
    b = ka.ka_batch_create(16)
    ka.ka_batch_set_option(b, ka.KA_BOPT_CACHE_BUDGET, budget)
    sims = []
    for spec, g in zip(BUDGET_MEMBERS, graphs):
        s = _make(spec, g)
        # one step per class, as in the step counts above (every class of this graph is
        # small, so by default its whole sweep would be one merged step)
        ka.ka_set_option(s, ka.KA_OPT_TAIL, 0)
        ka.ka_batch_add(b, s, spec[7])
        sims.append(s)
    assert graphs[2].C * 3 == 45
    left = ka.ka_batch_steps_left(b)
    assert left == expected_steps
    ka.ka_batch_run(b, left)
    assert ka.ka_batch_steps_left(b) == 0
    done = set()
    deadline = time.time() + 60
    while len(done) < len(BUDGET_MEMBERS):
        assert time.time() < deadline, "members did not complete in the projected steps"
        done.update(ka.ka_batch_poll(b))
        time.sleep(0.001)
    for k, (s, ref) in enumerate(zip(sims, solo)):
        for x, y in zip(ka.ka_get_state(s), ref):
            assert np.array_equal(np.asarray(x), np.asarray(y)), k
    b.free()
    for s in sims:
        s.free()


def test_cache_budget_set_before_members(graphs):
    b = ka.ka_batch_create(4)
    s = _make(MEMBERS[0], graphs[0])
    ka.ka_batch_add(b, s, 1)
    for opt in (ka.KA_BOPT_CACHE_BUDGET, ka.KA_BOPT_SOLO_BYTES):
        with pytest.raises(ka.KaError) as e:
            ka.ka_batch_set_option(b, opt, 1 << 20)
        assert e.value.code == ka.KA_ESTATE
        with pytest.raises(ka.KaError) as e:
            ka.ka_batch_set_option(b, opt, -1)
        assert e.value.code == ka.KA_EINVAL
    b.free()
    s.free()


def _working_set(spec, g):
    return 2 * g.N * (spec[5] // 64) * 8      # n and f


# 64 KiB: the 2D L=64 x 64, 3D L=16 x 128 and RRG N=1000 x 320 members run one at a time;
# 1 byte: every member does; 0: none does.
@pytest.mark.parametrize("solo_bytes", [1 << 16, 1, 0])
def test_solo_members_equal_solo(graphs, solo, solo_bytes):
    """KA_BOPT_SOLO_BYTES: members whose n and f take at least that many bytes skip the step
    kernel and run one at a time, in the order added, through their own pass kernels, one
    launch per step.  ka_batch_steps_left projects that schedule exactly (the solo members'
    steps add up, the others run from step 0), that many steps complete every member, and
    each ends in its solo state."""
    import time
    _say(f"batch: solo bytes {solo_bytes}")
    b = ka.ka_batch_create(64)
    ka.ka_batch_set_option(b, ka.KA_BOPT_SOLO_BYTES, solo_bytes)
    ka.ka_batch_set_option(b, ka.KA_BOPT_GRAPH_STEPS, 8)
    sims, batched, solo_steps, n_solo = [], 0, 0, 0
    for spec, g in zip(MEMBERS, graphs):
        s = _make(spec, g)
        if spec[0] == "rrg":
            ka.ka_set_option(s, ka.KA_OPT_TAIL, 0)   # one step per class
        ka.ka_batch_add(b, s, spec[7])
        sims.append(s)
        steps = g.C * spec[7]
        if solo_bytes > 0 and _working_set(spec, g) >= solo_bytes:
            solo_steps += steps
            n_solo += 1
        else:
            batched = max(batched, steps)
    assert n_solo == {1 << 16: 3, 1: len(MEMBERS), 0: 0}[solo_bytes]
    left = ka.ka_batch_steps_left(b)
    assert left == max(batched, solo_steps)
    # in uneven chunks, so that runs of step kernels and solo launches end mid-sweep
    chunks = [5, 17, 64, 3]
    q = 0
    while left > 0:
        r = min(left, chunks[q % len(chunks)])
        ka.ka_batch_run(b, r)
        left -= r
        q += 1
    assert ka.ka_batch_steps_left(b) == 0
    done = set()
    deadline = time.time() + 60
    while len(done) < len(MEMBERS):
        assert time.time() < deadline, "members did not complete in the projected steps"
        done.update(ka.ka_batch_poll(b))
        time.sleep(0.001)
    _assert_same([ka.ka_get_state(s) for s in sims], solo)
    assert all(s.t == spec[7] for s, spec in zip(sims, MEMBERS))
    b.free()
    for s in sims:
        s.free()


TAIL_MEMBERS = [
    # colourings ending in tiny classes: 17 classes, the last 4 (415, 104, 12, 1 edges)
    # merged; 11 classes, the last 3 merged; 22 classes, the last 3 merged
    ("rrg", 16384, 4, 2, 0.6, 64, 51, 3),
    ("rrg", 8192, 3, 1, 0.55, 128, 52, 4),
    ("rrg", 16384, 5, 3, 0.7, 192, 53, 2),
    ("rrg", 2000, 4, 2, 0.65, 128, 54, 3),      # every class small: one step per sweep
    ("lat", (3, 12), 6, 3, 0.8, 64, 55, 2),
]


def _tail_first(class_sizes, most=512):
    """First class of the trailing run of classes with at most `most` edges each, or the
    class count if that run holds fewer than two classes."""
    C = len(class_sizes)
    c = C
    while c > 0 and class_sizes[c - 1] <= most:
        c -= 1
    return c if C - c >= 2 else C


def test_solo_members_in_plane_groups():
    """A solo member whose word planes run in groups (KA_OPT_PLANE_GROUPS, as ka_sweep does
    for lattices beyond the Infinity Cache) advances group by group through each run of steps;
    lattices with word pairs and single words and a graph whose whole sweep is one merged
    launch, next to a member in the step kernel, all end in their solo states."""
    import time
    _say("batch: solo members in plane groups")
    specs = [  # graph, m, rho, R, seed, sweeps, planes per group
        (ka.ka_graph_lattice(2, 64), 2, 0.7, 256, 61, 3, 1),      # 2 planes of word pairs
        (ka.ka_graph_lattice(3, 16), 3, 0.85, 192, 62, 2, 2),     # 3 planes: groups of 2 and 1
        (ka.ka_graph_rrg(2000, 4, 63), 2, 0.65, 192, 63, 4, 2),   # every class small: one launch per sweep
        (ka.ka_graph_lattice(2, 8), 2, 0.6, 64, 64, 9, -1),       # 1 KiB: in the step kernel
    ]
    ref = []
    for g, m, rho, R, seed, n, grp in specs:
        s = ka.ka_init(g, m, rho, seed, R)
        ka.ka_set_option(s, ka.KA_OPT_PLANE_GROUPS, grp)
        ka.ka_sweep(s, n)
        ref.append(ka.ka_get_state(s))
        s.free()
    b = ka.ka_batch_create(8)
    ka.ka_batch_set_option(b, ka.KA_BOPT_SOLO_BYTES, 64 << 10)
    ka.ka_batch_set_option(b, ka.KA_BOPT_GRAPH_STEPS, 8)
    sims = []
    for g, m, rho, R, seed, n, grp in specs:
        s = ka.ka_init(g, m, rho, seed, R)
        ka.ka_set_option(s, ka.KA_OPT_PLANE_GROUPS, grp)
        ka.ka_batch_add(b, s, n)
        sims.append(s)
    left = ka.ka_batch_steps_left(b)
    chunks = [7, 30, 2, 64]
    q = 0
    while left > 0:
        r = min(left, chunks[q % len(chunks)])
        ka.ka_batch_run(b, r)
        left -= r
        q += 1
    done = set()
    deadline = time.time() + 60
    while len(done) < len(specs):
        assert time.time() < deadline, "members did not complete in the projected steps"
        done.update(ka.ka_batch_poll(b))
        time.sleep(0.001)
    for k, (s, r) in enumerate(zip(sims, ref)):
        for x, y in zip(ka.ka_get_state(s), r):
            assert np.array_equal(np.asarray(x), np.asarray(y)), k
    b.free()
    for s in sims:
        s.free()


def test_solo_members_with_no_sweeps():
    """Solo members queued behind one with no sweeps still start: the one with no sweeps ends
    at the step it starts, and the next starts there too."""
    _say("batch: solo members with zero sweeps in the queue")
    g = ka.ka_graph_lattice(2, 16)
    plan = [(1, 2), (2, 0), (3, 0), (4, 3)]      # (seed, sweeps)
    ref = []
    for seed, n in plan:
        s = ka.ka_init(g, 2, 0.6, seed, 64)
        ka.ka_sweep(s, n)
        ref.append(ka.ka_get_state(s))
        s.free()
    b = ka.ka_batch_create(8)
    ka.ka_batch_set_option(b, ka.KA_BOPT_SOLO_BYTES, 1)
    sims = []
    for seed, n in plan:
        s = ka.ka_init(g, 2, 0.6, seed, 64)
        ka.ka_batch_add(b, s, n)
        sims.append(s)
    assert ka.ka_batch_steps_left(b) == g.C * 5
    ka.ka_batch_wait_all(b)
    for k, (s, r) in enumerate(zip(sims, ref)):
        assert s.t == plan[k][1]
        for x, y in zip(ka.ka_get_state(s), r):
            assert np.array_equal(np.asarray(x), np.asarray(y)), k
    b.free()
    for s in sims:
        s.free()


@pytest.mark.parametrize("tail,all_solo", [(1, False), (0, False), (1, True)])
def test_batch_merged_tail_classes(tail, all_solo):
    """A graph member whose colouring ends in tiny classes runs that trailing run as one step
    (one workgroup per plane takes the classes in order), unless KA_OPT_TAIL is 0 on the sim;
    the projected steps count the run once, and either way every member ends in its solo
    state.  With every member run one at a time (KA_BOPT_SOLO_BYTES = 1) the merged run is one
    launch of the member's own tail kernel, and the steps add up."""
    _say(f"batch: merged tail classes, tail={tail}, all solo={all_solo}")
    graphs = [_graph(spec) for spec in TAIL_MEMBERS]
    solo = []
    for spec, g in zip(TAIL_MEMBERS, graphs):
        s = _make(spec, g)
        ka.ka_sweep(s, spec[7])
        solo.append(ka.ka_get_state(s))
        s.free()
    b = ka.ka_batch_create(8)
    if all_solo:
        ka.ka_batch_set_option(b, ka.KA_BOPT_SOLO_BYTES, 1)
    sims, expected = [], 0
    for spec, g in zip(TAIL_MEMBERS, graphs):
        s = _make(spec, g)
        ka.ka_set_option(s, ka.KA_OPT_TAIL, tail)
        ka.ka_batch_add(b, s, spec[7])
        sims.append(s)
        steps_per_sweep = g.C
        if spec[0] == "rrg" and tail:
            _, _, _, ec = ka.ka_graph_export(g)
            first = _tail_first(np.bincount(ec, minlength=g.C))
            assert first <= g.C - 2
            steps_per_sweep = first + 1
        if all_solo:
            expected += steps_per_sweep * spec[7]
        else:
            expected = max(expected, steps_per_sweep * spec[7])
    assert ka.ka_batch_steps_left(b) == expected
    ka.ka_batch_wait_all(b)
    for k, (s, ref) in enumerate(zip(sims, solo)):
        for x, y in zip(ka.ka_get_state(s), ref):
            assert np.array_equal(np.asarray(x), np.asarray(y)), k
    b.free()
    for s in sims:
        s.free()
