"""The autotuner's cache: a cached choice is applied to the context on a
cache hit exactly as a fresh tuning run applies it (CPU, stub context)."""
from paper_2605_30342_amd import scenes
from paper_2605_30342_amd.autotune import Autotuner, workload_class


class StubContext:
    device = 0

    def __init__(self):
        self.tuning = {"vis_batch": 64, "uq_batch": 256}
        self.set_calls = 0

    def get_tuning(self):
        return dict(self.tuning)

    def set_tuning(self, vis_batch=64, uq_batch=256):
        self.tuning = {"vis_batch": vis_batch, "uq_batch": uq_batch}
        self.set_calls += 1


class StubScene:
    n = 200_000


def test_cache_hit_applies_the_cached_choice(tmp_path):
    cams = scenes.sphere_cameras(4, 11, width=64, height=64)
    path = tmp_path / "tune.json"
    t = Autotuner(StubContext(), str(path))
    t.table[workload_class("query", StubScene.n, cams)] = {"uq_batch": 128, "ms": {}}
    t.table[workload_class("build", StubScene.n, cams)] = {"vis_batch": 256, "ms": {}}
    t.save()
    ctx = StubContext()
    t2 = Autotuner(ctx, str(path))          # loads the saved table
    r = t2.tune_query(StubScene(), None, 2, 8, cams, None, None)
    assert r["uq_batch"] == 128 and ctx.tuning == {"vis_batch": 64, "uq_batch": 128}

    class P:
        sh_degree = 2
    r = t2.tune_build(StubScene(), cams, P(), None, None)
    assert r["vis_batch"] == 256 and ctx.tuning == {"vis_batch": 256, "uq_batch": 128}


def test_apply_reports_a_miss():
    cams = scenes.sphere_cameras(2, 12, width=32, height=32)
    ctx = StubContext()
    assert not Autotuner(ctx).apply("query", 10, cams)
    assert ctx.set_calls == 0
