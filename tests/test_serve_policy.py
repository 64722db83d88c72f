"""CPU tests of the serving admission policy (no GPU): FIFO order, every limit
respected, head-of-line blocking instead of reordering, oversize first request."""
from collections import deque

from paper_2603_11531_amd.serve import form_batch


class R:
    def __init__(self, rid, n, t, b, p):
        self.rid, self.fp = rid, (n, t, b, p)


def fp(r):
    return r.fp


def test_fifo_and_request_limit():
    q = deque(R(i, 100, 10, 1000, 50) for i in range(10))
    b = form_batch(q, fp, max_batch=4, max_gaussians=10**9, max_tiles=10**9, capacity=10**9,
                   image_budget=10**9, image_in_use=0)
    assert [r.rid for r in b] == [0, 1, 2, 3] and [r.rid for r in q][:1] == [4]


def test_each_limit_stops_the_batch_at_the_head():
    for kw, stop in ((dict(max_gaussians=250), 2), (dict(max_tiles=25), 2), (dict(capacity=120), 2),
                     (dict(image_budget=2500), 2)):
        limits = dict(max_batch=64, max_gaussians=10**9, max_tiles=10**9, capacity=10**9, image_budget=10**9)
        limits.update(kw)
        q = deque(R(i, 100, 10, 1000, 50) for i in range(6))
        b = form_batch(q, fp, image_in_use=0, **limits)
        assert len(b) == stop, kw
        assert q[0].rid == stop


def test_no_reordering_behind_a_request_that_does_not_fit():
    q = deque([R(0, 100, 10, 1000, 50), R(1, 10**6, 10, 1000, 50), R(2, 1, 1, 1, 1)])
    b = form_batch(q, fp, max_batch=8, max_gaussians=1000, max_tiles=10**9, capacity=10**9,
                   image_budget=10**9, image_in_use=0)
    assert [r.rid for r in b] == [0] and [r.rid for r in q] == [1, 2]


def test_memory_in_use_counts_and_oversize_first_request():
    q = deque([R(0, 100, 10, 1000, 10**12)])
    b = form_batch(q, fp, max_batch=8, max_gaussians=10**9, max_tiles=10**9, capacity=100,
                   image_budget=10**9, image_in_use=0)
    assert [r.rid for r in b] == [0]           # pair estimate above capacity: admitted alone
    q = deque([R(1, 100, 10, 1000, 1)])
    assert form_batch(q, fp, max_batch=8, max_gaussians=10**9, max_tiles=10**9, capacity=100,
                      image_budget=1500, image_in_use=600) == []
    assert len(q) == 1


# ---------------------------------------------------------------- the server loop on a simulated device
class _FakeSlot:
    """A batch slot whose batch takes `overhead` + the sum of its requests' costs of simulated time."""

    def __init__(self, be):
        self.be, self.requests = be, []

    def launch(self, reqs, registry):
        self.requests = list(reqs)
        self.t_start = self.be.t
        self.t_end = self.t_start + self.be.overhead + sum(self.be.cost(r) for r in reqs)
        self.be.batches.append([r.rid for r in reqs])

    def ready(self):
        return self.be.t >= self.t_end

    def overflowed(self):
        return False

    def rendered(self):
        return True


class _FakeBackend:
    """Simulated device and clock: time advances only when the server sleeps."""
    device = None

    def __init__(self, cost, overhead=1e-3):
        self.t, self.cost, self.overhead, self.batches = 0.0, cost, overhead, []

    def new_slot(self, *limits):
        return _FakeSlot(self)

    def start(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, seconds):
        self.t += max(seconds, 1e-6)

    def image(self, W, H):
        return None

    def slot_times(self, slot):
        return slot.t_start, slot.t_end

    def render_alone(self, registry, r):
        self.t += self.cost(r)

    def finish(self):
        pass


def _server(timeout_s=None, n_slots=1, max_batch=2):
    import mgs_data
    from paper_2603_11531_amd import serve

    class _Scene:
        n = 1000

    registry = {"a": (_Scene(), None)}
    be = _FakeBackend(cost=lambda r: 0.010)
    srv = serve.Server(registry, max_batch=max_batch, max_gaussians=10**9, max_tiles=10**9, capacity=10**12,
                       n_slots=n_slots, image_budget_bytes=10**12, timeout_s=timeout_s, backend=be)
    cam = mgs_data.look_at((0.0, 0.0, -4.0), width=64, height=48, f=64.0)
    reqs = [serve.Request(rid=k, scene="a", cam=cam, arrival=0.001 * k) for k in range(20)]
    return srv, be, reqs


def test_server_loop_fifo_batches_on_a_simulated_device():
    srv, be, reqs = _server()
    served = srv.run(reqs)
    assert sorted(r.rid for r in served) == list(range(20)) and not srv.timed_out
    flat = [rid for b in be.batches for rid in b]
    assert flat == list(range(20)) and max(len(b) for b in be.batches) == 2      # FIFO, batches of <= 2
    assert all(r.done >= r.start >= r.arrival for r in served)


def test_request_timeout_cancels_requests_queued_too_long():
    """A burst the device cannot keep up with (21 ms per batch of two, arrivals every 1 ms): with
    a 30 ms timeout the oldest queued requests are cancelled, none is both served and cancelled,
    and every served request started within the timeout of its arrival."""
    srv, be, reqs = _server(timeout_s=0.030)
    served = srv.run(reqs)
    ids_s, ids_t = {r.rid for r in served}, {r.rid for r in srv.timed_out}
    assert ids_t and ids_s and not (ids_s & ids_t) and ids_s | ids_t == set(range(20))
    assert all(r.path == "timed out" for r in srv.timed_out)
    assert all(r.start - r.arrival <= 0.030 + 1e-3 for r in served)
    assert all(be.t >= r.arrival + 0.030 for r in srv.timed_out)


def test_duration_leaves_the_late_queue_unserved():
    srv, be, reqs = _server()
    served = srv.run(reqs, duration=0.035)
    assert served and srv.unserved
    assert {r.rid for r in served} | {r.rid for r in srv.unserved} == {r.rid for r in reqs if r.arrival <= 0.035}
    assert all(r.start <= 0.035 for r in served)
