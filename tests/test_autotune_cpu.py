"""The launch-shape autotuner's host logic with a stand-in context: candidate
shapes, the batch key, the search picking the fastest shape, and the cache."""
import json

from paper_1501_05630_amd import autotune


class FakeCtx:
    def __init__(self, metas):
        self.meta = dict(enumerate(metas))
        self.cfg = None
        self.applied = []

    def icm_set_run_config(self, **cfg):
        self.cfg = dict(cfg)
        self.applied.append(dict(cfg))


def fake_timer(ctx, handles, sweeps):
    c = ctx.cfg
    # fastest at 512 threads, 16 slots, 256-sweep launches
    return (abs(c["threads"] - 512) / 256 + abs(c["icm_slots"] - 16) / 8
            + (0 if c["sweeps_per_launch"] == 256 else 0.5) + 1.0)


META = dict(N=512, K=20, R=4, Kc=14, jkind=1)


def test_candidates_respect_four_moves_per_wave():
    c = autotune.candidates()
    assert c and all(x["icm_slots"] <= 4 * (x["threads"] // 64) for x in c)
    assert all(x["use_graph"] == 1 for x in c)
    assert {x["threads"] for x in c} == {64, 128, 256, 512, 1024}
    assert len(c) == len({json.dumps(x, sort_keys=True) for x in c})


def test_batch_key_counts_shapes():
    k1 = autotune.batch_key([META] * 1000, 1000)
    k2 = autotune.batch_key([META] * 1024, 1024)
    assert k1 == k2                                   # same power-of-two bucket
    k3 = autotune.batch_key([META] * 512 + [dict(META, N=64)] * 512, 1024)
    assert k3 != k2 and "N64_" in k3 and "N512_" in k3


def test_search_picks_the_fastest_and_caches_it(tmp_path):
    cache = str(tmp_path / "tune.json")
    ctx = FakeCtx([META] * 8)
    best, info = autotune.tune(ctx, list(range(8)), cache_path=cache, timer=fake_timer)
    assert best == dict(threads=512, icm_slots=16, sweeps_per_launch=256, use_graph=1,
                        class_threads=[-1, -1, -1, -1])
    assert info["source"] == "search" and ctx.cfg == best
    assert len(info["ms_per_sweep"]) == len(autotune.candidates())
    with open(cache) as f:
        assert json.load(f)[info["key"]] == best
    # a second batch of the same shape takes the cached choice without timing
    ctx2 = FakeCtx([META] * 8)

    def no_timer(*a):
        raise AssertionError("cached shapes are not timed again")

    best2, info2 = autotune.tune(ctx2, list(range(8)), cache_path=cache, timer=no_timer)
    assert best2 == best and info2["source"] == "cache" and ctx2.applied == [best]


def test_restricted_candidates_and_no_cache():
    ctx = FakeCtx([META] * 4)
    cands = [c for c in autotune.candidates() if c["sweeps_per_launch"] == 128]
    best, info = autotune.tune(ctx, [0, 1, 2, 3], cache_path=None, cands=cands, timer=fake_timer)
    assert best["sweeps_per_launch"] == 128 and best["threads"] == 512 and best["icm_slots"] == 16


def test_several_size_classes_get_their_own_thread_counts():
    # a batch of 64-site and 2000-site units (size classes 0 and 2): after the
    # common search each class's thread count is refined on the whole batch
    ctx = FakeCtx([dict(META, N=64)] * 4 + [dict(META, N=2000)] * 4)

    def timer(ctx, handles, sweeps):
        c = ctx.cfg
        ct = c["class_threads"]
        small = ct[0] if ct[0] > 0 else c["threads"]
        large = ct[2] if ct[2] > 0 else c["threads"]
        return abs(small - 128) / 64 + abs(large - 1024) / 64 + abs(c["icm_slots"] - 16) / 8

    best, info = autotune.tune(ctx, list(range(8)), cache_path=None, timer=timer)
    assert best["class_threads"][0] == 128 and best["class_threads"][2] == 1024
    assert best["class_threads"][1] == -1 and best["class_threads"][3] == -1
    assert ctx.cfg == best
    # the common search plus every thread count for each of the two classes
    assert len(info["ms_per_sweep"]) <= len(autotune.candidates()) + 2 * len(autotune.THREADS)
    assert autotune.size_classes(ctx.meta.values()) == [0, 2]
