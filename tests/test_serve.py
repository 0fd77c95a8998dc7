"""Scheduling logic of the continuous-batching server on the CPU, with a
simulated backend (virtual clock, memory sizes, completion times, failures)."""
import numpy as np
import pytest

from paper_2605_30342_amd import scenes
from paper_2605_30342_amd.serve import (CANCELLED, DONE, FAILED, REJECTED, BackendError, Server)


class FakeBackend:
    """Batch duration = fixed + per-view time; workspace = per-view bytes.
    Scores are deterministic per (scene, camera) so mixing can be checked."""

    def __init__(self, bytes_per_view=100, t_fixed=1.0, t_view=0.1, fail_plan=(), fail_launch=(), stuck=(),
                 scene_bytes_per_view=None, fail_after=None):
        self.t = 0.0
        self.bpv = bytes_per_view
        self.scene_bpv = dict(scene_bytes_per_view or {})
        self.fail_after = fail_after          # (scene, n): launches of that scene after the n-th fail
        self.t_fixed, self.t_view = t_fixed, t_view
        self.fail_plan, self.fail_launch, self.stuck = set(fail_plan), set(fail_launch), set(stuck)
        self.launches = []
        self.live = {}

    def now(self):
        return self.t

    def wait(self, dt):
        self.t += max(dt, 0.01)

    def plan_bytes(self, scene_id, cams_list, limit=None):
        if scene_id in self.fail_plan:
            raise BackendError("plan failed")
        return self.scene_bpv.get(scene_id, self.bpv) * sum(c.n for c in cams_list)

    def launch(self, scene_id, cams_list, slot, nbytes):
        if scene_id in self.fail_launch:
            raise BackendError("out of memory")
        assert slot not in self.live, "slot reused while busy"
        nv = sum(c.n for c in cams_list)
        if self.fail_after is not None and scene_id == self.fail_after[0]:
            if sum(s == scene_id for s, _, _ in self.launches) >= self.fail_after[1]:
                raise BackendError("out of memory")
        h = {"slot": slot, "end": self.t + self.t_fixed + self.t_view * nv,
             "scores": np.concatenate([self.score(scene_id, c) for c in cams_list]), "scene": scene_id}
        self.live[slot] = h
        self.launches.append((scene_id, nv, slot))
        return h

    def done(self, h):
        if h["scene"] in self.stuck:
            return False
        return self.t >= h["end"]

    def result(self, h):
        return h["scores"]

    def release(self, h):
        self.live.pop(h["slot"], None)

    @staticmethod
    def score(scene_id, cams):
        return cams.K[:, 0].astype(np.float64) * 0 + cams.t[:, 0] * 1000 + hash(scene_id) % 97


def cams(n, seed):
    return scenes.room_candidates(n, seed, ((0, 6), (0, 4), (0, 3)), 32, 24)


def test_all_requests_complete_with_their_own_scores():
    be = FakeBackend()
    srv = Server(be, memory_budget=10_000, n_slots=2, max_batch_views=64)
    rids = [srv.submit(f"s{i % 3}", cams(4 + i % 5, i)) for i in range(20)]
    srv.run_until_idle(timeout=1e4)
    for i, rid in enumerate(rids):
        r = srv.requests[rid]
        assert r.status == DONE
        np.testing.assert_array_equal(r.scores, FakeBackend.score(f"s{i % 3}", r.cams))
        assert r.latency >= be.t_fixed


def test_same_scene_requests_are_merged_and_different_scenes_overlap():
    be = FakeBackend()
    srv = Server(be, memory_budget=100_000, n_slots=2, max_batch_views=64)
    for i in range(6):
        srv.submit("A", cams(4, i))
    srv.submit("B", cams(4, 99))
    srv.step()
    # first batch: all six A requests merged; second slot: scene B concurrently
    assert be.launches[0] == ("A", 24, 0)
    assert be.launches[1] == ("B", 4, 1)
    assert srv.merged_requests == 5
    srv.run_until_idle(timeout=1e4)
    assert all(r.status == DONE for r in srv.requests.values())


def test_admission_respects_the_memory_budget():
    be = FakeBackend(bytes_per_view=100)
    srv = Server(be, memory_budget=1000, n_slots=4, max_batch_views=64)
    for i in range(4):
        srv.submit(f"s{i}", cams(6, i))        # 600 bytes each: only one fits at a time
    srv.step()
    assert len(srv.running) == 1 and srv.in_use == 600
    peak = 0
    while not srv.idle():
        srv.step()
        peak = max(peak, srv.in_use)
        assert srv.in_use <= 1000
        be.wait(0.05)
    assert peak == 600
    assert all(r.status == DONE for r in srv.requests.values())


def test_large_head_request_is_not_starved():
    be = FakeBackend(bytes_per_view=100)
    srv = Server(be, memory_budget=1000, n_slots=4, max_batch_views=64)
    srv.submit("small0", cams(2, 0))
    srv.submit("big", cams(9, 1))               # 900 bytes: needs the memory of everything else
    for i in range(5):
        srv.submit(f"small{i + 1}", cams(2, 10 + i))
    srv.run_until_idle(timeout=1e4)
    order = [s for s, _, _ in be.launches]
    assert order.index("big") == 1               # admitted right after the head, before later smalls
    assert srv.requests[1].status == DONE


def test_request_whose_single_view_exceeds_the_budget_is_rejected_and_others_proceed():
    be = FakeBackend(bytes_per_view=100, scene_bytes_per_view={"x": 600})
    srv = Server(be, memory_budget=500, n_slots=2)
    big = srv.submit("x", cams(8, 0))
    ok = srv.submit("y", cams(2, 1))
    srv.run_until_idle(timeout=1e4)
    assert srv.requests[big].status == REJECTED
    assert srv.requests[ok].status == DONE
    assert not any(s == "x" for s, _, _ in be.launches)
    assert srv.in_use == 0 and not srv.pending


def test_request_above_the_budget_is_served_in_chunks_of_its_views():
    """8 views of 100 bytes against a 500-byte budget: halved into two
    chunks of 4 views, run one after the other; the request gets the scores
    of all its views in order, and counts once in the statistics."""
    be = FakeBackend(bytes_per_view=100)
    srv = Server(be, memory_budget=500, n_slots=2)
    c = cams(8, 0)
    big = srv.submit("x", c)
    ok = srv.submit("y", cams(2, 1))
    srv.run_until_idle(timeout=1e4)
    r = srv.requests[big]
    assert r.status == DONE and r.latency > 0
    np.testing.assert_array_equal(r.scores, FakeBackend.score("x", c))
    assert [nv for s, nv, _ in be.launches if s == "x"] == [4, 4]
    assert srv.requests[ok].status == DONE
    st = srv.stats()
    assert st["requests_done"] == 2 and st["views_done"] == 10 and st["split_requests"] == 1
    assert srv.in_use == 0 and not srv.pending


def test_uneven_request_is_halved_until_every_chunk_fits():
    """13 views of 100 bytes against a 300-byte budget: 13 is halved into 6
    and 7, those into chunks of 3, 3, 3 and 4, the 4 into 2 and 2; the
    scores land at their views' positions, and the request is running from
    its first chunk on."""
    be = FakeBackend(bytes_per_view=100)
    srv = Server(be, memory_budget=300, n_slots=3)
    c = cams(13, 3)
    rid = srv.submit("x", c)
    srv.step()
    assert srv.requests[rid].status == "running"
    srv.run_until_idle(timeout=1e4)
    r = srv.requests[rid]
    assert r.status == DONE
    np.testing.assert_array_equal(r.scores, FakeBackend.score("x", c))
    sizes = [nv for _, nv, _ in be.launches]
    assert sum(sizes) == 13 and max(sizes) <= 3
    assert srv.in_use <= 300


def test_failed_chunk_fails_its_request_and_drops_its_other_chunks():
    """The second chunk's launch fails: the request fails, no further chunk
    of it runs, and other requests proceed."""
    be = FakeBackend(bytes_per_view=100, fail_after=("x", 1))
    srv = Server(be, memory_budget=400, n_slots=1)
    big = srv.submit("x", cams(12, 0))                # chunks 3, 3, 3, 3
    ok = srv.submit("y", cams(2, 1))
    srv.run_until_idle(timeout=1e4)
    assert srv.requests[big].status == FAILED
    assert [nv for s, nv, _ in be.launches if s == "x"] == [3]
    assert srv.requests[ok].status == DONE
    assert srv.in_use == 0 and not srv.pending and sorted(srv.free_slots) == [0]


def test_split_request_cannot_be_cancelled_once_a_chunk_runs():
    be = FakeBackend(bytes_per_view=100)
    srv = Server(be, memory_budget=400, n_slots=1)
    big = srv.submit("x", cams(8, 0))
    srv.step()
    assert not srv.cancel(big)
    srv.run_until_idle(timeout=1e4)
    assert srv.requests[big].status == DONE


def test_backend_failures_fail_only_their_requests():
    be = FakeBackend(fail_plan={"bad_plan"}, fail_launch={"oom"})
    srv = Server(be, memory_budget=10_000, n_slots=2)
    a = srv.submit("bad_plan", cams(2, 0))
    b = srv.submit("oom", cams(2, 1))
    c = srv.submit("good", cams(2, 2))
    srv.run_until_idle(timeout=1e4)
    assert srv.requests[a].status == FAILED and srv.requests[b].status == FAILED
    assert srv.requests[c].status == DONE
    assert srv.in_use == 0 and sorted(srv.free_slots) == [0, 1]


def test_cancel_pending_request():
    be = FakeBackend()
    srv = Server(be, memory_budget=10_000, n_slots=1)
    a = srv.submit("A", cams(2, 0))
    b = srv.submit("B", cams(2, 1))
    srv.step()                                   # A runs on the only slot, B pending
    assert srv.cancel(b)
    assert not srv.cancel(a)                     # running requests cannot be cancelled
    srv.run_until_idle(timeout=1e4)
    assert srv.requests[a].status == DONE and srv.requests[b].status == CANCELLED


def test_stuck_batch_times_out_without_freeing_its_slot():
    be = FakeBackend(stuck={"stuck"})
    srv = Server(be, memory_budget=10_000, n_slots=2, stuck_timeout=5.0)
    a = srv.submit("stuck", cams(2, 0))
    b = srv.submit("fine", cams(2, 1))
    for _ in range(1000):
        srv.step()
        be.wait(0.05)
        if srv.requests[a].status == FAILED and srv.requests[b].status == DONE:
            break
    assert srv.requests[a].status == FAILED and srv.requests[a].error == "timed out"
    assert srv.requests[b].status == DONE
    assert len(srv.running) == 1                 # the stuck batch still holds its slot


def test_latency_stats():
    be = FakeBackend()
    srv = Server(be, memory_budget=10_000, n_slots=2)
    for i in range(10):
        srv.submit("A" if i % 2 else "B", cams(3, i), t_arrival=0.0)
    srv.run_until_idle(timeout=1e4)
    st = srv.stats()
    assert st["requests_done"] == 10 and st["views_done"] == 30
    assert st["p50_latency_ms"] <= st["p99_latency_ms"]
    assert st["views_per_s"] > 0


# ---------------------------------------------------------------- GPU backend planning, on the CPU

class _Plan:
    def __init__(self, n, rec, ins):
        self.max_records, self.max_instances = rec, ins
        self.bytes = 1000 + 10 * rec + 20 * ins + n


class _StubCtx:
    """Stands in for api.Context: exact sizing returns 100 records and 300
    instances per view of 32x24 and twice that for 64x48; allocation
    optionally refuses."""
    device = 0

    def __init__(self, refuse_alloc=False):
        self.exact_calls = []
        self.allocs = 0
        self.refuse = refuse_alloc

    def query_plan_exact(self, dsc, cams, params, sh_degree, stream=None):
        f = np.where(cams.wh[:, 0] == 32, 1, 2)
        self.exact_calls.append(cams.n)
        return _Plan(dsc.n, int(100 * f.sum()), int(300 * f.sum()))

    def query_plan(self, dsc, cams, sh_degree, max_records, max_instances):
        return _Plan(dsc.n, max_records, max_instances)

    def alloc_workspace(self, plan):
        import torch
        self.allocs += 1
        if self.refuse:
            raise torch.cuda.OutOfMemoryError("no memory")
        return object()


class _Dsc:
    n = 1000


def _gpu_backend(ctx):
    from paper_2605_30342_amd.serve import GpuBackend
    be = GpuBackend(ctx, n_slots=2, params=object(), slack=1.5)
    be._streams = [None] * 3          # no device streams on the CPU
    be.add_scene("A", _Dsc(), None, 2, 4)
    return be


def _cams_wh(n, w, h, seed):
    return scenes.room_candidates(n, seed, ((0, 6), (0, 4), (0, 3)), w, h)


def test_gpu_backend_plans_on_the_host_after_one_exact_pass_per_image_size():
    """Admission sizing allocates nothing; each (scene, image size) is sized
    exactly once, later batches from the learnt per-view rates with slack;
    a mixed batch adds the rates of its sizes."""
    ctx = _StubCtx()
    be = _gpu_backend(ctx)
    b1 = be.plan_bytes("A", [_cams_wh(4, 32, 24, 1)])
    assert ctx.exact_calls == [4] and ctx.allocs == 0
    b2 = be.plan_bytes("A", [_cams_wh(4, 32, 24, 2), _cams_wh(2, 32, 24, 3)])
    assert ctx.exact_calls == [4] and ctx.allocs == 0      # known size: no device pass
    assert be.rates[("A", 32, 24)] == [100.0, 300.0]
    p = be._plan("A", _cams_wh(6, 32, 24, 4))
    assert p.max_records >= 6 * 100 * 1.5 and p.max_instances >= 6 * 300 * 1.5
    assert b2 > b1
    from paper_2605_30342_amd.scenes import Cameras
    mixed = Cameras.concat([_cams_wh(3, 32, 24, 5), _cams_wh(2, 64, 48, 6)])
    p = be._plan("A", mixed)
    assert ctx.exact_calls == [4, 2]                      # only the new size is sized exactly
    assert p.max_records >= (3 * 100 + 2 * 200) * 1.5


def test_gpu_backend_learns_larger_counts_from_completed_batches():
    ctx = _StubCtx()
    be = _gpu_backend(ctx)
    c = _cams_wh(4, 32, 24, 1)
    be.plan_bytes("A", [c])
    be._learn("A", c, 4 * 150, 4 * 280)          # a batch that needed more records, fewer instances
    assert be.rates[("A", 32, 24)] == [150.0, 300.0]


def test_gpu_backend_turns_allocation_failure_into_a_failed_request():
    """The workspace is allocated at launch, after admission; an allocation
    the device refuses fails the batch's requests instead of escaping the
    server loop."""
    ctx = _StubCtx(refuse_alloc=True)
    be = _gpu_backend(ctx)
    srv = Server(be, memory_budget=1 << 40, n_slots=2, max_batch_views=16)
    rid = srv.submit("A", _cams_wh(3, 32, 24, 1))
    srv.step()
    r = srv.requests[rid]
    assert r.status == FAILED and "allocation" in r.error
    assert srv.in_use == 0 and sorted(srv.free_slots) == [0, 1]


def test_gpu_backend_sizes_exactly_when_the_estimate_exceeds_the_free_budget():
    """An estimate (rates x slack) above the free memory is replaced by the
    exact size, computed once and reused while the batch waits and at its
    launch."""
    ctx = _StubCtx()
    be = _gpu_backend(ctx)
    c = _cams_wh(4, 32, 24, 1)
    est = be.plan_bytes("A", [c])
    assert ctx.exact_calls == [4]
    exact = _Plan(1000, 400, 1200).bytes
    assert est > exact
    assert be.plan_bytes("A", [c], limit=exact) == exact
    assert ctx.exact_calls == [4, 4]
    assert be.plan_bytes("A", [c], limit=exact) == exact       # cached: no second pass
    assert ctx.exact_calls == [4, 4]


def test_merged_batches_keep_to_a_slots_share_of_memory():
    """Followers join the head's batch only while the batch's workspace stays
    within budget / slots, so that the slots can run batches side by side."""
    be = FakeBackend(bytes_per_view=100)
    srv = Server(be, memory_budget=10_000, n_slots=2, max_batch_views=512)
    for i in range(10):
        srv.submit("A", cams(8, i))
    srv.step()
    assert len(be.launches) == 2                        # both slots busy
    assert all(nv * 100 <= 5_000 for _, nv, _ in be.launches)
    assert be.launches[0][1] == 48                       # six requests of 8 views
    srv.run_until_idle(timeout=1e4)
    assert all(r.status == DONE for r in srv.requests.values())
