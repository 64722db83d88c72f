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
