"""Host-side tests of the continuous-batching scheduler against a fake
executor with a programmable latency model (no GPU)."""
import numpy as np
import pytest

from paper_2202_05977_amd import serve


class VClock:
    """Virtual time: advances a tick on every read, and jumps on sleep."""

    def __init__(self, tick=1e-5):
        self.t = 0.0
        self.tick = tick

    def __call__(self):
        self.t += self.tick
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeExecutor(serve.Executor):
    def __init__(self, clock, per_px=1e-9, fixed=50e-6, fail_on=None, bytes_per_px=100):
        self.clock = clock
        self.per_px = per_px
        self.fixed = fixed
        self.fail_on = fail_on or set()
        self.bytes_per_px = bytes_per_px
        self.inflight = {}
        self.launches = []
        self.max_used = 0
        self.n = 0

    def workspace_bytes(self, reqs):
        return sum(r.H * r.W * self.bytes_per_px for r in reqs) + 256

    def launch(self, reqs, slot, ws_offset=0):
        self.n += 1
        if self.n in self.fail_on:
            raise RuntimeError("injected failure")
        # serialised device: starts after the previous batch ends
        start = max([self.clock.t] + [t for t, _ in self.inflight.values()])
        done = start + self.fixed + self.per_px * sum(r.H * r.W for r in reqs)
        tok = self.n
        self.inflight[tok] = (done, self.workspace_bytes(reqs))
        self.max_used = max(self.max_used, sum(b for _, b in self.inflight.values()))
        self.launches.append([r.rid for r in reqs])
        return tok

    def done(self, tok):
        if self.inflight[tok][0] <= self.clock.t:
            del self.inflight[tok]
            return True
        return False


@pytest.fixture(autouse=True)
def virtual_sleep(monkeypatch):
    holder = {}

    def fake_sleep(dt):
        holder["clock"].sleep(dt)
    monkeypatch.setattr(serve.time, "sleep", fake_sleep)
    return holder


def trace(n_streams=16, frames=20, rate=2000.0, seed=3):
    return serve.poisson_trace(n_streams, frames, rate, ((36, 64), (72, 128), (144, 256)), seed)


def test_trace_shape():
    sizes, reqs = serve.poisson_trace(64, 300, 2000.0, ((360, 640), (720, 1280)), seed=7)
    assert len(reqs) == 64 * 300 and len(sizes) == 64
    t = np.array([r.t_arrival for r in reqs])
    assert np.all(np.diff(t) >= 0)
    # aggregate rate close to 2000/s while every stream is still active
    assert 1900 < np.sum(t < 5.0) / 5.0 < 2100


def test_all_complete_with_batching_and_order(virtual_sleep):
    clock = VClock()
    virtual_sleep["clock"] = clock
    _, reqs = trace(rate=4000.0)
    ex = FakeExecutor(clock, per_px=2e-8)
    st = serve.Server(ex, budget_bytes=1 << 40, clock=clock).run(reqs)
    assert st.frames == len(reqs) and st.errors == 0
    for r in reqs:
        assert r.t_arrival <= r.t_start <= r.t_done
    # under load batches hold more than one frame
    assert st.mean_batch > 1.0
    # oldest first: starts are ordered like arrivals
    starts = np.array([r.t_start for r in sorted(reqs, key=lambda r: r.t_arrival)])
    assert np.all(np.diff(starts) >= 0)


def test_continuous_admission_overlaps_inflight_work(virtual_sleep):
    """A request that arrives while one batch runs is launched before that
    batch completes (second slot), i.e. work overlaps on the device."""
    clock = VClock()
    virtual_sleep["clock"] = clock
    a = serve.Request(0, 0, 0.0, 72, 128)
    b = serve.Request(1, 1, 1e-4, 72, 128)
    ex = FakeExecutor(clock, per_px=1e-7)    # ~0.9 ms per frame
    serve.Server(ex, 1 << 40, max_inflight=2, clock=clock).run([a, b])
    assert b.t_start < a.t_done
    assert len(ex.launches) == 2


def test_budget_is_respected_and_oversize_rejected(virtual_sleep):
    clock = VClock()
    virtual_sleep["clock"] = clock
    _, reqs = trace(rate=8000.0)
    ex = FakeExecutor(clock, per_px=2e-8)
    one_big = 144 * 256 * 100 + 256
    budget = 3 * one_big
    huge = serve.Request(len(reqs), 99, 0.001, 720, 1280)   # larger than the budget
    st = serve.Server(ex, budget, clock=clock).run(reqs + [huge])
    assert ex.max_used <= budget
    assert huge.error == "budget"
    assert st.errors == 1 and st.frames == len(reqs)


def test_executor_failure_errors_the_batch_and_continues(virtual_sleep):
    clock = VClock()
    virtual_sleep["clock"] = clock
    _, reqs = trace(rate=2000.0)
    ex = FakeExecutor(clock, fail_on={2})
    st = serve.Server(ex, 1 << 40, clock=clock).run(reqs)
    failed = [r for r in reqs if r.error]
    assert failed and all(r.error.startswith("launch") for r in failed)
    assert st.frames == len(reqs) - len(failed) > 0
    assert all(np.isfinite(r.t_done) for r in reqs)


def test_fifo_single_is_serial(virtual_sleep):
    clock = VClock()
    virtual_sleep["clock"] = clock
    _, reqs = trace(n_streams=4, frames=10, rate=500.0)

    class Blocking(FakeExecutor):
        def wait(self, tok):
            clock.t = max(clock.t, self.inflight[tok][0])
            del self.inflight[tok]

    ex = Blocking(clock)
    st = serve.fifo_single(ex, reqs, clock=clock)
    assert st.mean_batch == 1.0 and st.frames == len(reqs)
    ordered = sorted(reqs, key=lambda r: r.t_arrival)
    for x, y in zip(ordered, ordered[1:]):
        assert y.t_start >= x.t_done


def test_arena_first_fit():
    a = serve.Arena(1024, align=256)
    o1 = a.alloc(300)        # 512
    o2 = a.alloc(256)
    assert (o1, o2) == (0, 512)
    assert a.alloc(512) is None
    a.free(o1)
    assert a.alloc(256) == 0
    assert a.used == 512


def test_per_stream_cap_bounds_frames_in_flight(virtual_sleep):
    """With a per-stream cap (the size of a stream's output ring), no stream
    ever has more frames in flight than the cap, even when one batch could
    take many of its frames, and each stream's frames still start in order."""
    clock = VClock()
    virtual_sleep["clock"] = clock
    _, reqs = trace(n_streams=4, frames=30, rate=20000.0)   # heavily overloaded
    ex = FakeExecutor(clock, per_px=2e-8)
    ex.per_stream_cap = 2
    srv = serve.Server(ex, 1 << 40, max_inflight=3, max_batch=64, clock=clock)
    st = srv.run(reqs)
    assert st.frames == len(reqs) and st.errors == 0
    assert srv.max_stream_inflight <= 2
    # over the whole run: at any launch, a stream's frames launched but not
    # done never exceed the cap
    for s in range(4):
        mine = sorted((r for r in reqs if r.stream == s), key=lambda r: r.seq)
        starts = [r.t_start for r in mine]
        assert starts == sorted(starts)
        for r in mine:
            overlapping = [q for q in mine if q.t_start <= r.t_start < q.t_done]
            assert len(overlapping) <= 2
    # without the cap the same load puts more frames of a stream in flight
    _, reqs2 = trace(n_streams=4, frames=30, rate=20000.0)
    srv2 = serve.Server(FakeExecutor(clock, per_px=2e-8), 1 << 40, max_inflight=3, max_batch=64,
                        clock=clock)
    srv2.run(reqs2)
    assert srv2.max_stream_inflight > 2


def test_trace_frame_index_per_stream():
    sizes, reqs = serve.poisson_trace(8, 12, 500.0, ((36, 64),), seed=1)
    for s in range(8):
        seqs = [r.seq for r in sorted((r for r in reqs if r.stream == s), key=lambda r: r.t_arrival)]
        assert seqs == list(range(12))
