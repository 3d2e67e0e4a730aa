"""Serving scheduler on the CPU with a fake backend and a fake clock:
admission never exceeds the HBM budget, batches group equal view sizes in
arrival order, oversized requests are rejected, failed launches release their
slot and budget."""
import pytest

from paper_2604_03748_amd import lnm
from paper_2604_03748_amd.serve import Request, Scheduler, poisson_requests


class FakeClock:
    def __init__(self, tick=1e-4):
        self.t, self.tick = 0.0, tick

    def __call__(self):
        self.t += self.tick
        return self.t


class Inst:
    def __init__(self, res):
        self.res = res


class FakeBackend:
    """Service time = 1 ms + 0.1 ms per request; bytes = res^2."""

    def __init__(self, clock, n_streams=2, fail_batches=()):
        self.clock = clock
        self.streams = list(range(n_streams))
        self.fail = set(fail_batches)
        self.launched = []
        self.busy = set()

    def request_bytes(self, res):
        return res * res

    def launch(self, slot, reqs, instances, keep_ids=()):
        k = len(self.launched)
        self.launched.append([r.rid for r in reqs])
        assert slot not in self.busy
        assert len({instances[r.instance].res for r in reqs}) == 1
        if k in self.fail:
            raise lnm.LnmError(lnm.LNM_ERR_DEVICE, "injected failure")
        self.busy.add(slot)
        return (slot, self.clock.t + 1e-3 + 1e-4 * len(reqs))

    def done(self, handle):
        if self.clock.t >= handle[1]:
            self.busy.discard(handle[0])
            return True
        return False


def test_budget_and_batching():
    clock = FakeClock()
    insts = {0: Inst(64), 1: Inst(128), 2: Inst(64)}
    reqs = poisson_requests(3, rate_hz=4000, duration_s=0.05, seed=3)
    be = FakeBackend(clock)
    budget = 5 * 128 * 128
    sch = Scheduler(be, insts, budget, max_batch=8, clock=clock)
    st = sch.run(reqs)
    assert st["requests"] == len(reqs) and st["rejected"] == 0 and st["failed"] == 0
    assert sch.peak_in_use <= budget
    assert st["p99_ms"] >= st["p50_ms"] > 0
    for r in sch.done:
        assert r.t_done >= r.t_admit >= r.t_arrival
    # batches keep arrival order within a view size
    for ids in be.launched:
        assert ids == sorted(ids)
    assert max(len(b) for b in be.launched) > 1  # batching happened


def test_oversized_request_is_rejected():
    clock = FakeClock()
    insts = {0: Inst(64), 1: Inst(512)}
    reqs = [Request(0, 0, 0, 0.0), Request(1, 1, 0, 0.0), Request(2, 0, 1, 0.001)]
    sch = Scheduler(FakeBackend(clock), insts, budget_bytes=100 * 100, clock=clock)
    st = sch.run(reqs)
    assert st["rejected"] == 1 and sch.rejected[0].rid == 1
    assert st["requests"] == 2


def test_failed_launch_releases_slot_and_budget():
    clock = FakeClock()
    insts = {0: Inst(32)}
    reqs = [Request(k, 0, k, 0.0002 * k) for k in range(40)]
    be = FakeBackend(clock, n_streams=1, fail_batches={0, 3})
    sch = Scheduler(be, insts, budget_bytes=4 * 32 * 32, max_batch=4, clock=clock)
    st = sch.run(reqs)
    assert st["failed"] > 0
    assert st["requests"] + st["failed"] == len(reqs)
    assert sch.in_use == 0 and len(sch.free_slots) == 1


def test_poisson_arrivals_rate():
    reqs = poisson_requests(64, rate_hz=2000, duration_s=2.0, seed=7)
    assert 3700 < len(reqs) < 4300
    assert all(0 <= r.instance < 64 for r in reqs)
    times = [r.t_arrival for r in reqs]
    assert times == sorted(times)
