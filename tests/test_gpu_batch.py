"""Ensembles in one persistent launch: every realization bit-identical to its
solo run (and to the oracle), under every launch configuration; admission by
arena budget; graph-captured solo runs."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_00310_amd as P

    P.lib()
    return P


def _reals():
    from paper_1606_00310_amd.batch import Realization as R

    return [
        R(64, 64, 0.5, 0.0, 37, 1001), R(128, 128, 0.75, 0.0, 23, 1002), R(256, 256, 0.9375, 0.0, 11, 1003),
        R(512, 512, 0.5, 0.0, 6, 1004), R(1024, 1024, 0.75, 0.0, 4, 1005), R(2048, 2048, 0.9375, 0.0, 3, 1006),
        R(4, 4, 0.5, 0.5, 50, 7), R(8, 32, 0.93, 0.07, 19, 8), R(4096, 16, 0.3, 0.0, 9, 9),
        R(8192, 8, 0.75, 0.25, 13, 10), R(32, 1024, 1.0, 0.0, 17, 11), R(128, 4, 0.5, 0.0, 0, 12),
        R(256, 64, 0.5, 0.0, 21, 13, True), R(64, 4096, 0.1875, 0.0, 8, 2**40 + 5), R(16, 16, 0.0, 1.0, 5, 14),
        R(512, 128, 0.9375, 0.0625, 12, 15),
        # rows of 16..64 words: temporally blocked passes when the configuration's depth is > 0
        R(2048, 512, 0.75, 0.25, 7, 16), R(4096, 256, 0.5, 0.0, 5, 17), R(8192, 128, 0.9375, 0.0625, 4, 18),
        R(2048, 64, 0.5, 0.0, 9, 19), R(8192, 32, 1.0, 0.0, 6, 20), R(2048, 1024, 0.93, 0.07, 3, 21),
        # two bands only: the first wave holds active and idle row groups (the idle ones compute on valid
        # rows and their stores are dropped), the other waves only take part in the barriers
        R(2048, 32, 0.5, 0.0, 9, 22), R(1024, 32, 0.75, 0.25, 7, 23),
    ]


def _solo(sca, r):
    lat = sca.Lattice(r.X, r.Y, seed=r.seed)
    lat.step(r.n_mcs, r.p, r.q, force_persite=r.force_persite)
    torch.cuda.synchronize()
    return lat


@pytest.fixture(scope="module")
def solo_states(sca):
    out = []
    for r in _reals():
        lat = _solo(sca, r)
        out.append((lat.slopes.clone(), lat.meta()[1], lat.roughness()))
        lat.close()
    return out


CONFIGS = [
    dict(block_threads=512, blocks_per_cu=2, lds_bytes=65536, order=0, words_per_lane=1, depth=2),
    dict(block_threads=256, blocks_per_cu=4, lds_bytes=65536, order=1, words_per_lane=2, depth=1),
    dict(block_threads=1024, blocks_per_cu=1, lds_bytes=0, order=0, words_per_lane=1, depth=0),
    dict(block_threads=1024, blocks_per_cu=1, lds_bytes=0, order=0, words_per_lane=2, depth=2),
    dict(block_threads=512, blocks_per_cu=1, lds_bytes=16384, order=1, words_per_lane=2, depth=0),
    dict(block_threads=256, blocks_per_cu=8, lds_bytes=4096, order=0, words_per_lane=1, depth=2),
    dict(block_threads=1024, blocks_per_cu=2, lds_bytes=0, order=0, words_per_lane=1, depth=1),
    # realizations with more work than the average per workgroup split over 2 or 4 workgroups
    dict(block_threads=1024, blocks_per_cu=1, lds_bytes=65536, order=0, words_per_lane=2, depth=2, max_parts=4),
    dict(block_threads=512, blocks_per_cu=2, lds_bytes=0, order=0, words_per_lane=1, depth=2, max_parts=2),
    dict(block_threads=256, blocks_per_cu=4, lds_bytes=0, order=0, words_per_lane=1, depth=1, max_parts=4),
    # 3- and 4-MCS passes: one 512-thread workgroup per CU
    dict(block_threads=512, blocks_per_cu=1, lds_bytes=65536, order=0, words_per_lane=1, depth=4),
    dict(block_threads=512, blocks_per_cu=1, lds_bytes=0, order=0, words_per_lane=2, depth=3, max_parts=4),
    dict(block_threads=512, blocks_per_cu=1, lds_bytes=0, order=1, words_per_lane=1, depth=4, max_parts=2),
]


def _cfg_id(c):
    return "b{block_threads}-c{blocks_per_cu}-l{lds_bytes}-o{order}-w{words_per_lane}-d{depth}".format(**c) + \
        (f"-p{c['max_parts']}" if "max_parts" in c else "")


@pytest.mark.parametrize("cfg", CONFIGS, ids=_cfg_id)
@pytest.mark.parametrize("epoch", [5, 1000])
def test_batch_equals_solo(sca, solo_states, cfg, epoch):
    from paper_1606_00310_amd.batch import Batch, state_bytes

    reals = _reals()
    _say(f"[batch] cfg={cfg} epoch={epoch}")
    arena = sum(state_bytes(r.X, r.Y) for r in reals)
    b = Batch(max_slots=len(reals), arena_bytes=arena, config=cfg)
    slots = b.admit(reals)
    while b.run(epoch):
        pass
    torch.cuda.synchronize()
    for r, s, (ref, h0, mom) in zip(reals, slots, solo_states):
        S, h = b.state(s)
        assert torch.equal(S, ref), r
        assert int(h[0]) == h0, r
        assert b.info(s).t == r.n_mcs
        assert b.roughness(s) == mom
    b.close()


def test_batch_matches_oracle(orc, sca):
    from paper_1606_00310_amd.batch import Batch, state_bytes

    reals = [r for r in _reals() if r.sites <= 1 << 18]
    b = Batch(max_slots=len(reals), arena_bytes=sum(state_bytes(r.X, r.Y) for r in reals))
    slots = b.admit(reals)
    while b.run(7):
        pass
    torch.cuda.synchronize()
    for r, s in zip(reals, slots):
        st = orc.flat(r.X, r.Y)
        orc.run(st, r.n_mcs, r.p, r.q, seed=r.seed, force_persite=r.force_persite)
        S, h = b.state(s)
        assert np.array_equal(S.cpu().numpy().view(np.uint64), orc.pack(st)), r
        assert int(h[0]) == st.h0
    b.close()


# One long realization among short ones: it has more work than the average
# per workgroup, so it runs split over 2 or 4 workgroups with barriers among
# them (bands of 8 or 16 rows).  Rows of 8, 16 and 32 words.
SPLIT_CASES = [
    (2048, 2048, 0.75, 0.0, 41, 1024, 2, 4),
    (2048, 256, 0.9375, 0.0625, 33, 256, 2, 2),
    (1024, 1024, 0.5, 0.0, 29, 512, 2, 4),
    (4096, 512, 1.0, 0.0, 23, 512, 1, 4),
    (2048, 1024, 0.5, 0.5, 18, 256, 2, 4),
    (2048, 2048, 0.5, 0.0, 37, 512, 4, 2),
    (4096, 1024, 0.9375, 0.0625, 21, 512, 3, 4),
]


@pytest.mark.parametrize("X,Y,p,q,n,bt,depth,parts", SPLIT_CASES)
def test_split_realization_equals_solo(sca, X, Y, p, q, n, bt, depth, parts):
    from paper_1606_00310_amd.batch import Batch, Realization as R, state_bytes

    _say(f"[split] {X}x{Y} p={p} q={q} n={n} block={bt} depth={depth} parts={parts}")
    long_one = R(X, Y, p, q, n, 5150 + X // 256 + Y)
    others = [R(64, 64, 0.5, 0.0, 3, 5200 + i) for i in range(4)] + [R(1024, 64, 0.75, 0.0, 2, 5210)]
    reals = [long_one] + others
    cfg = dict(block_threads=bt, blocks_per_cu=1 if depth > 2 else 1024 // bt, lds_bytes=0, order=0,
               words_per_lane=1, depth=depth, max_parts=parts)
    b = Batch(max_slots=len(reals), arena_bytes=sum(state_bytes(r.X, r.Y) for r in reals), config=cfg)
    slots = b.admit(reals)
    for epoch in (n // 3, n):   # two epochs: the counters restart at each launch
        b.run(epoch)
    while b.run(n):
        pass
    torch.cuda.synchronize()
    for r, s in zip(reals, slots):
        lat = _solo(sca, r)
        S, h = b.state(s)
        assert torch.equal(S, lat.slopes), r
        assert int(h[0]) == lat.meta()[1], r
        assert b.roughness(s) == lat.roughness(), r
        lat.close()
    b.close()


def test_split_realization_matches_oracle(orc, sca):
    """A 1024 x 1024 realization split over four workgroups, from the flat
    surface, against the oracle."""
    from paper_1606_00310_amd.batch import Batch, Realization as R, state_bytes

    reals = [R(1024, 1024, 0.75, 0.25, 11, 6101), R(64, 64, 0.5, 0.0, 2, 6102)]
    cfg = dict(block_threads=256, blocks_per_cu=4, lds_bytes=0, order=0, words_per_lane=1, depth=2, max_parts=4)
    b = Batch(max_slots=2, arena_bytes=sum(state_bytes(r.X, r.Y) for r in reals), config=cfg)
    slots = b.admit(reals)
    while b.run(11):
        pass
    torch.cuda.synchronize()
    for r, s in zip(reals, slots):
        st = orc.flat(r.X, r.Y)
        orc.run(st, r.n_mcs, r.p, r.q, seed=r.seed)
        S, h = b.state(s)
        assert np.array_equal(S.cpu().numpy().view(np.uint64), orc.pack(st)), r
        assert int(h[0]) == st.h0
    b.close()


@pytest.mark.parametrize("depth,parts", [(4, 1), (3, 2), (4, 4)])
def test_deep_batch_passes_match_oracle(orc, sca, depth, parts):
    """3- and 4-MCS blocked passes of the persistent kernel (one 512-thread
    workgroup per CU), whole and split, from the flat surface, against the
    oracle: 16- and 8-word rows, q > 0 and an odd number of draws."""
    from paper_1606_00310_amd.batch import Batch, Realization as R, state_bytes

    reals = [R(2048, 512, 0.75, 0.25, 13, 6201), R(1024, 1024, 0.5, 0.0, 10, 6202), R(64, 64, 0.5, 0.0, 2, 6203)]
    cfg = dict(block_threads=512, blocks_per_cu=1, lds_bytes=0, order=0, words_per_lane=1, depth=depth,
               max_parts=parts)
    _say(f"[batch] deep passes depth={depth} parts={parts}")
    b = Batch(max_slots=len(reals), arena_bytes=sum(state_bytes(r.X, r.Y) for r in reals), config=cfg)
    slots = b.admit(reals)
    while b.run(13):
        pass
    torch.cuda.synchronize()
    for r, s in zip(reals, slots):
        st = orc.flat(r.X, r.Y)
        orc.run(st, r.n_mcs, r.p, r.q, seed=r.seed)
        S, h = b.state(s)
        assert np.array_equal(S.cpu().numpy().view(np.uint64), orc.pack(st)), r
        assert int(h[0]) == st.h0
    b.close()


def test_deep_batch_passes_need_one_512_thread_workgroup_per_cu(sca):
    from paper_1606_00310_amd import ScaError
    from paper_1606_00310_amd.batch import Batch, state_bytes

    for cfg in (dict(block_threads=1024, blocks_per_cu=1, depth=3), dict(block_threads=512, blocks_per_cu=2, depth=4),
                dict(block_threads=512, blocks_per_cu=1, depth=5)):
        full = dict(lds_bytes=0, order=0, words_per_lane=1, max_parts=1, **cfg)
        with pytest.raises(ScaError):
            Batch(max_slots=1, arena_bytes=state_bytes(64, 64), config=full)


def test_admission_budget_and_reuse(sca):
    from paper_1606_00310_amd import ScaError
    from paper_1606_00310_amd.batch import Batch, Realization as R, state_bytes

    big = R(1024, 1024, 0.5, 0.0, 3, 1)
    small = R(64, 64, 0.5, 0.0, 5, 2)
    b = Batch(max_slots=4, arena_bytes=2 * state_bytes(1024, 1024))
    s1 = b.admit([big])
    assert b.try_admit([big, big]) is None          # all or none: not enough arena
    s2 = b.admit([big])
    assert b.try_admit([small]) is None              # arena full
    b.release(s1[0])
    s3 = b.admit([small, small, small])              # slots 4 in total now used: big + 3 small
    assert b.try_admit([small]) is None              # no slot left
    with pytest.raises(ScaError):
        b.admit([R(100, 64, 0.5, 0.0, 1, 1)])        # invalid size
    while b.run(2):
        pass
    lat = sca.Lattice(64, 64, seed=2)
    lat.step(5, 0.5)
    for s in s3:
        assert torch.equal(b.state(s)[0], lat.slopes)
    ref_big = sca.Lattice(1024, 1024, seed=1)
    ref_big.step(3, 0.5)
    assert torch.equal(b.state(s2[0])[0], ref_big.slopes)
    b.close()


def test_late_admission_matches_solo(sca):
    """Realizations admitted while others are mid-run end bit-identical to
    their solo runs (the continuous-batching case)."""
    from paper_1606_00310_amd.batch import Batch, Realization as R, state_bytes

    first = [R(256, 256, 0.75, 0.0, 40, 100 + i) for i in range(3)]
    late = [R(128, 512, 0.9375, 0.0, 25, 200 + i) for i in range(3)]
    b = Batch(max_slots=8, arena_bytes=sum(state_bytes(r.X, r.Y) for r in first + late))
    s_first = b.admit(first)
    b.run(10)
    b.run(10)
    s_late = b.admit(late)
    while b.run(10):
        pass
    torch.cuda.synchronize()
    for r, s in zip(first + late, s_first + s_late):
        assert torch.equal(b.state(s)[0], _solo(sca, r).slopes), r
    b.close()


@pytest.mark.parametrize("X,Y,p,q", [(64, 64, 0.5, 0.0), (2048, 2048, 0.9375, 0.0), (512, 32, 0.93, 0.07)])
def test_graph_step_equals_plain(sca, X, Y, p, q):
    a = sca.Lattice(X, Y, seed=77)
    b = sca.Lattice(X, Y, seed=77)
    a.step(33, p, q)
    b.step(33, p, q, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(a.slopes, b.slopes) and a.meta() == b.meta()


def test_serving_mix_equals_alone(sca):
    """Requests arriving while others run are admitted as slots free up; every
    served realization equals its solo run bit for bit."""
    from paper_1606_00310_amd import serve
    from paper_1606_00310_amd.batch import Batch, Realization as R, state_bytes

    reqs = []
    seed = 900
    sizes = [(64, 3), (256, 1), (128, 2), (512, 1), (64, 4), (1024, 1), (32, 2), (256, 2)]
    for i, (L, k) in enumerate(sizes):
        rs = []
        for j in range(k):
            rs.append(R(L, L, (0.5, 0.75, 0.9375)[(i + j) % 3], 0.0, 15 + 7 * ((i * 3 + j) % 5), seed))
            seed += 1
        reqs.append(serve.Request(i, rs, arrival=0.0005 * i))
    budget = state_bytes(1024, 1024) + 4 * state_bytes(256, 256)   # forces waiting
    b = Batch(max_slots=6, arena_bytes=budget)
    srv = serve.Server(serve.BatchBackend(b), mcs_epoch=6)
    done = srv.serve(reqs)
    assert len(done) == len(reqs)
    for req in done:
        for r, res in zip(req.realizations, req.results):
            lat = _solo(sca, r)
            assert torch.equal(res["slopes"], lat.slopes), r
            assert res["h0"] == lat.meta()[1]
            assert res["moments"] == lat.roughness()
    b.close()


def test_work_quota_epochs_equal_solo(sca, solo_states):
    from paper_1606_00310_amd.batch import Batch, state_bytes

    reals = _reals()
    b = Batch(max_slots=len(reals), arena_bytes=sum(state_bytes(r.X, r.Y) for r in reals))
    slots = b.admit(reals)
    epochs = 0
    while b.run_work(3 * 256 * 256):
        epochs += 1
    assert epochs > 1
    torch.cuda.synchronize()
    for r, s, (ref, h0, mom) in zip(reals, slots, solo_states):
        S, h = b.state(s)
        assert torch.equal(S, ref), r
        assert int(h[0]) == h0
    b.close()


def test_autotune_small(sca):
    """The autotuner times each candidate on the sample, checks that all of
    them leave the same states, and returns the fastest."""
    from paper_1606_00310_amd import autotune
    from paper_1606_00310_amd.batch import Realization as R

    sample = [R(2048, 256, 0.75, 0.0, 6, 300), R(64, 64, 0.5, 0.0, 9, 301), R(1024, 1024, 0.9375, 0.0625, 5, 302)]
    cands = [autotune.CANDIDATES[0], autotune.CANDIDATES[2], autotune.CANDIDATES[-1]]
    best, table = autotune.autotune(sample, candidates=cands, cache_path=None)
    assert best in cands and len(table) == 3 and all(t > 0 for _, t in table)
