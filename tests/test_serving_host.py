"""Host logic of the serving request loop (no GPU): requests arriving over
time are admitted per size-class lane in arrival order as slots free up, every
request is served exactly once, admission happens while a round is in flight
(the request joins the next round), and lanes progress independently.

The lanes here are stand-ins with the server's protocol (submit / launch /
wait / poll / stats) whose rounds take a fixed host time; the request loop is
the one the bench runs."""
import collections
import time

import numpy as np

from paper_1705_06073_amd import serving


class FakeResult:
    def __init__(self, tag, rounds):
        self.tag = tag
        self.rounds = rounds


class FakeLane:
    """`slots` requests at once; request `tag` needs rounds_of(tag) rounds; a
    round takes `dt` seconds of host time from launch."""

    def __init__(self, slots, dt, rounds_of):
        self.slots, self.dt, self.rounds_of = slots, dt, rounds_of
        self.admitted = []          # admission order
        self.pending = []           # admitted since the last launch
        self.running = {}           # tag -> rounds left
        self.done = collections.deque()
        self.in_flight = False
        self.t_ready = 0.0
        self.rounds = 0
        self.joined_mid_round = 0
        self.max_held = 0

    def submit(self, ptr, n, tag):
        assert ptr == 1000 + tag
        if len(self.running) + len(self.pending) >= self.slots:
            return False
        if self.in_flight:
            self.joined_mid_round += 1
        self.pending.append(tag)
        self.admitted.append(tag)
        self.max_held = max(self.max_held, len(self.running) + len(self.pending))
        return True

    def launch(self):
        if self.in_flight or not (self.running or self.pending):
            return
        for t in self.pending:
            self.running[t] = self.rounds_of(t)
        self.pending = []
        self.in_flight = True
        self.t_ready = time.perf_counter() + self.dt

    def wait(self, block=True):
        if not self.in_flight:
            return True, 0
        if time.perf_counter() < self.t_ready:
            if not block:
                return False, 0
            time.sleep(self.t_ready - time.perf_counter())
        self.in_flight = False
        self.rounds += 1
        fin = 0
        for t in list(self.running):
            self.running[t] -= 1
            if self.running[t] == 0:
                del self.running[t]
                self.done.append(FakeResult(t, self.rounds_of(t)))
                fin += 1
        return True, fin

    def poll(self):
        out = list(self.done)
        self.done.clear()
        return out

    def stats(self):
        return dict(in_flight=len(self.running) + len(self.pending), rounds=self.rounds)


def test_request_loop_serves_every_request_in_arrival_order_per_lane():
    rng = np.random.default_rng(3)
    R = 300
    classes = ((1024, 6), (16384, 3))
    sizes = rng.choice(np.array([256, 1024, 4096, 16384]), size=R)
    arrivals = np.sort(rng.uniform(0.0, 0.15, R))
    lane_of = [serving.lane_index(classes, int(n)) for n in sizes]
    lanes = [FakeLane(6, 0.0004, lambda t: 2 + t % 5),
             FakeLane(3, 0.0010, lambda t: 3 + t % 4)]
    res, lat, st = serving.run_stream(lanes, lane_of, arrivals, sizes, lambda i: 1000 + i)
    assert all(r is not None for r in res)
    assert [r.tag for r in res] == list(range(R))
    assert np.all(np.isfinite(lat)) and np.all(lat > 0)
    for li, lane in enumerate(lanes):
        mine = [i for i in range(R) if lane_of[i] == li]
        assert lane.admitted == mine           # FIFO per lane
        assert lane.max_held <= lane.slots     # never more than its slots
        assert not lane.running and not lane.pending
    # requests served by the slow lane wait at least their rounds
    for i in range(R):
        if lane_of[i] == 1:
            assert lat[i] >= (3 + i % 4) * 0.0010 * 0.99
    assert sum(l.joined_mid_round for l in lanes) > 0  # admission did not wait for rounds
    summ = serving.summarize(lat, sizes, arrivals, st["wall_s"])
    assert summ["requests"] == R and set(summ["by_n"]) == {"256", "1024", "4096", "16384"}


def test_lane_index_by_size_class():
    classes = ((1024, 8), (4096, 4), (65536, 2))
    assert serving.lane_index(classes, 2) == 0
    assert serving.lane_index(classes, 1024) == 0
    assert serving.lane_index(classes, 1025) == 1
    assert serving.lane_index(classes, 65536) == 2
    try:
        serving.lane_index(classes, 65537)
    except ValueError:
        pass
    else:
        raise AssertionError("no lane should take n > 65536")
