"""The autotuner's cache: a cached choice is applied to the context on a
cache hit exactly as a fresh tuning run applies it (CPU, stub context)."""
from paper_2605_30342_amd import scenes
from paper_2605_30342_amd.autotune import CANDIDATES, DEFAULT, TIE, Autotuner, pick, workload_class


class StubContext:
    device = 0

    def __init__(self):
        self.tuning = {"vis_batch": 64, "uq_batch": 256, "vis_order": 0, "uq_order": 0}
        self.set_calls = 0

    def get_tuning(self):
        return dict(self.tuning)

    def set_tuning(self, vis_batch=64, uq_batch=256, vis_order=0, uq_order=0):
        self.tuning = {"vis_batch": vis_batch, "uq_batch": uq_batch, "vis_order": vis_order, "uq_order": uq_order}
        self.set_calls += 1


class StubScene:
    n = 200_000


def test_candidates_cover_both_axes():
    assert {b for b, _ in CANDIDATES} == {64, 128, 256} and {o for _, o in CANDIDATES} == {0, 1, 2, 3, 4}
    assert len(CANDIDATES) == 15


def test_cache_hit_applies_the_cached_choice(tmp_path):
    cams = scenes.sphere_cameras(4, 11, width=64, height=64)
    path = tmp_path / "tune.json"
    t = Autotuner(StubContext(), str(path))
    t.table[workload_class("query", StubScene.n, cams)] = {"uq_batch": 128, "uq_order": 1, "ms": {}}
    t.table[workload_class("build", StubScene.n, cams)] = {"vis_batch": 256, "vis_order": 1, "ms": {}}
    t.save()
    ctx = StubContext()
    t2 = Autotuner(ctx, str(path))          # loads the saved table
    r = t2.tune_query(StubScene(), None, 2, 8, cams, None, None)
    assert r["uq_batch"] == 128
    assert ctx.tuning == {"vis_batch": 64, "uq_batch": 128, "vis_order": 0, "uq_order": 1}

    class P:
        sh_degree = 2
    r = t2.tune_build(StubScene(), cams, P(), None, None)
    assert r["vis_batch"] == 256
    assert ctx.tuning == {"vis_batch": 256, "uq_batch": 128, "vis_order": 1, "uq_order": 1}


def test_entries_without_an_order_take_order_zero(tmp_path):
    cams = scenes.sphere_cameras(4, 11, width=64, height=64)
    ctx = StubContext()
    ctx.tuning["uq_order"] = 1
    t = Autotuner(ctx)
    t.table[workload_class("query", StubScene.n, cams)] = {"uq_batch": 64, "ms": {}}
    assert t.apply("query", StubScene.n, cams)
    assert ctx.tuning["uq_batch"] == 64 and ctx.tuning["uq_order"] == 0


def test_apply_reports_a_miss():
    cams = scenes.sphere_cameras(2, 12, width=32, height=32)
    ctx = StubContext()
    assert not Autotuner(ctx).apply("query", 10, cams)
    assert ctx.set_calls == 0


def test_default_schedule_wins_ties_within_the_noise_margin():
    """A candidate replaces the default only when faster by more than TIE."""
    d = DEFAULT["build"]
    times = {c: 3.0 for c in CANDIDATES}
    times[(64, 0)] = 2.8721
    times[d] = 2.8722                      # equal within run-to-run noise
    assert pick(times, d) == d
    times[d] = 2.8721 * (1 + 2 * TIE)      # clearly slower
    assert pick(times, d) == (64, 0)
    assert pick({(128, 1): 1.0, (64, 0): 2.0}, d) == (128, 1)   # default not timed
