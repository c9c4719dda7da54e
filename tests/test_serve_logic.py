"""Host logic of the serving loop (admission in arrival order by budget,
whole requests only, retirement and latency accounting), with a fake batch
backend on the CPU."""
import pytest

from paper_1606_00310_amd.batch import Realization as R
from paper_1606_00310_amd.serve import Request, Server, latency_stats


class FakeBackend:
    """Slots and an arena budget; run() advances every admitted realization."""

    def __init__(self, max_slots, budget):
        self.max_slots, self.budget = max_slots, budget
        self.used = {}        # slot -> [real, t]
        self.runs = []

    def _bytes(self, r):
        return r.X * r.Y // 4 + 8

    def try_admit(self, reals):
        free_slots = [s for s in range(self.max_slots) if s not in self.used]
        need = sum(self._bytes(r) for r in reals)
        have = self.budget - sum(self._bytes(v[0]) for v in self.used.values())
        if len(reals) > len(free_slots) or need > have:
            return None
        slots = free_slots[:len(reals)]
        for s, r in zip(slots, reals):
            self.used[s] = [r, 0]
        return slots

    def run(self, epoch):
        active = 0
        for v in self.used.values():
            left = v[0].n_mcs - v[1]
            if left > 0:
                v[1] += min(left, epoch)
                active += 1
        self.runs.append(active)
        return active

    def run_work(self, quota):
        active = 0
        for v in self.used.values():
            left = v[0].n_mcs - v[1]
            if left > 0:
                v[1] += min(left, max(1, quota // (v[0].X * v[0].Y)))
                active += 1
        self.runs.append(active)
        return active

    def sync(self):
        pass

    def finished(self, slot):
        r, t = self.used[slot]
        return t >= r.n_mcs

    def collect(self, slot):
        r, t = self.used[slot]
        return {"t": t, "seed": r.seed}

    def release(self, slot):
        del self.used[slot]


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.001
        return self.t


def _req(i, *sizes, mcs=10):
    return Request(i, [R(L, L, 0.5, 0.0, mcs, 100 * i + k) for k, L in enumerate(sizes)])


def test_fifo_admission_and_completion():
    be = FakeBackend(max_slots=4, budget=10**9)
    srv = Server(be, mcs_epoch=4, clock=Clock())
    reqs = [_req(0, 64, 64), _req(1, 128), _req(2, 64, 64, 64), _req(3, 32)]
    for r in reqs:
        srv.submit(r)
    while srv.queue or srv.running:
        srv.step()
    assert [r.rid for r in srv.completed][:2] == [0, 1]
    assert len(srv.completed) == 4
    for r in reqs:
        assert [x["t"] for x in r.results] == [10] * len(r.realizations)
        assert [x["seed"] for x in r.results] == [x.seed for x in r.realizations]
        assert r.latency is not None and r.latency > 0
    # request 2 (three slots) had to wait for slots freed by 0 and 1
    assert reqs[2].admitted > reqs[0].admitted
    assert not be.used


def test_whole_requests_only_and_head_of_line():
    be = FakeBackend(max_slots=8, budget=3 * (64 * 64 // 4 + 8))
    srv = Server(be, mcs_epoch=5, clock=Clock())
    srv.submit(_req(0, 64, 64))
    srv.submit(_req(1, 64, 64))      # does not fit next to request 0
    srv.submit(_req(2, 64))          # would fit, but waits behind request 1
    srv.step()
    assert set(srv.running) == {0}
    assert [r.rid for r in srv.queue] == [1, 2]
    while srv.queue or srv.running:
        srv.step()
    assert [r.rid for r in srv.completed] == [0, 1, 2]


def test_request_that_never_fits_is_reported():
    be = FakeBackend(max_slots=2, budget=10**9)
    srv = Server(be, clock=Clock())
    srv.submit(_req(0, 64, 64, 64))
    with pytest.raises(RuntimeError):
        srv.step()


def test_zero_mcs_request_completes_without_running():
    be = FakeBackend(max_slots=2, budget=10**9)
    srv = Server(be, clock=Clock())
    srv.submit(_req(0, 64, mcs=0))
    srv.step()
    assert len(srv.completed) == 1 and be.runs == []


def test_serve_with_arrivals_and_stats():
    be = FakeBackend(max_slots=3, budget=10**9)
    srv = Server(be, mcs_epoch=3, clock=Clock())
    reqs = [_req(i, 64, mcs=7) for i in range(10)]
    for i, r in enumerate(reqs):
        r.arrival = 0.002 * i
    done = srv.serve(reqs)
    assert len(done) == 10
    st = latency_stats(done)
    assert st["n"] == 10 and st["p50_s"] <= st["p99_s"] <= st["max_s"]


def test_work_quota_finishes_small_lattices_first():
    be = FakeBackend(max_slots=4, budget=10**9)
    srv = Server(be, clock=Clock(), work_quota=64 * 64 * 50)
    srv.submit(Request(0, [R(256, 256, 0.5, 0.0, 40, 1)]))
    srv.submit(Request(1, [R(64, 64, 0.5, 0.0, 40, 2)]))
    srv.step()
    # the 64x64 realization covers all 40 MCS in the first epoch, the 256x256 one 3
    assert [r.rid for r in srv.completed] == [1]
    while srv.running:
        srv.step()
    assert srv.completed[-1].results[0]["t"] == 40
