"""Admission policy of the serving loop, host logic only (CPU): first-in
first-out, a bounded bypass of a head that does not fit, no starvation, and
refused requests failing alone."""
from paper_1410_1942_amd.serve import ADMITTED, BUSY, REFUSED, AdmissionQueue


class FakeArena:
    """Room for `budget` units and `slots` solves; a request is its size,
    negative sizes are invalid (refused)."""

    def __init__(self, budget, slots=100):
        self.free, self.slots, self.log = budget, slots, []

    def __call__(self, r):
        if r < 0:
            self.log.append(("refused", r))
            return REFUSED
        if r > self.free or self.slots == 0:
            return BUSY
        self.free -= r
        self.slots -= 1
        self.log.append(("admitted", r))
        return ADMITTED

    def release(self, r):
        self.free += r
        self.slots += 1


def _queue(items, **kw):
    q = AdmissionQueue(**kw)
    for r in items:
        q.push(r)
    return q


def test_fifo_when_everything_fits():
    q = _queue([3, 1, 4, 1, 5])
    out = q.admit(FakeArena(100))
    assert [r for r, _ in out] == [3, 1, 4, 1, 5] and len(q) == 0


def test_stops_at_budget_in_order_without_bypass():
    q = _queue([4, 4, 4], lookahead=0)
    a = FakeArena(9)
    out = q.admit(a)
    assert [r for r, _ in out] == [4, 4] and list(q.q) == [4]


def test_small_requests_pass_a_blocked_head():
    q = _queue([50, 2, 3, 60, 1], lookahead=8, max_bypass=16)
    a = FakeArena(10)
    out = q.admit(a)
    # the head (50) does not fit; 2, 3 and 1 go first, 60 waits behind it
    assert [r for r, _ in out] == [2, 3, 1]
    assert list(q.q) == [50, 60] and q.passed == 3


def test_lookahead_limits_how_far_behind_the_head():
    q = _queue([50, 60, 70, 1], lookahead=2)
    out = q.admit(FakeArena(10))
    assert out == [] and list(q.q) == [50, 60, 70, 1]


def test_bypass_is_bounded_then_the_head_goes_first():
    q = _queue([50] + [1] * 10, lookahead=20, max_bypass=4)
    a = FakeArena(1000 - 990)            # room for small ones only
    out = q.admit(a)
    assert [r for r, _ in out] == [1, 1, 1, 1] and q.passed == 4
    # more room, but the head still does not fit: nothing else passes it
    a.free += 5
    assert q.admit(a) == []
    # room for the head: it goes first, then the queue flows again
    a.free += 100
    out = q.admit(a)
    assert [r for r, _ in out][0] == 50 and q.passed == 0


def test_refused_requests_fail_alone_and_do_not_count_as_passing():
    q = _queue([-1, 2, 50, -3, 4], lookahead=8, max_bypass=1)
    a = FakeArena(10)
    out = q.admit(a)
    assert out[0] == (-1, REFUSED) and out[1] == (2, ADMITTED)
    # behind the blocked head 50: -3 refused (does not count), 4 admitted (counts)
    assert (-3, REFUSED) in out and (4, ADMITTED) in out
    assert list(q.q) == [50] and q.passed == 1


def test_released_room_admits_the_head():
    q = _queue([6, 6, 6], lookahead=0)
    a = FakeArena(12)
    assert [r for r, _ in q.admit(a)] == [6, 6]
    a.release(6)
    assert [r for r, _ in q.admit(a)] == [6] and len(q) == 0
