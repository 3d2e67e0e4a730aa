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


class Tensor:
    """Stand-in for a device tensor: only its size matters to the scheduler."""

    def __init__(self, nbytes):
        self.n = nbytes

    def numel(self):
        return self.n // 4

    def element_size(self):
        return 4


class GridInst(Inst):
    def __init__(self, res, grid_bytes, brick_bytes):
        super().__init__(res)
        self.density = Tensor(grid_bytes)
        self.bricks = Tensor(brick_bytes) if brick_bytes else None


class ResidentBackend(FakeBackend):
    @staticmethod
    def resident_bytes(inst):
        n = inst.density.numel() * 4
        return n + (inst.bricks.numel() * 4 if inst.bricks is not None else 0)


def test_resident_grids_and_bricks_are_charged():
    clock = FakeClock()
    # grids 4000 / 8000 / 16000 B with brick copies twice as large; budget 40000
    insts = {0: GridInst(32, 4000, 8000), 1: GridInst(32, 8000, 16000), 2: GridInst(32, 16000, 32000)}
    budget = 40000
    be = ResidentBackend(clock)
    sch = Scheduler(be, insts, budget, max_batch=4, clock=clock)
    # grids 28000, then bricks smallest first: 8000 fits (36000), 16000 and 32000 do not
    assert sch.resident == 36000 and sch.in_use == 36000
    assert sorted(sch.dropped_bricks) == [1, 2] and insts[1].bricks is None and insts[0].bricks is not None
    reqs = [Request(k, k % 3, k, 0.0001 * k) for k in range(30)]
    st = sch.run(reqs)
    assert st["requests"] == 30 and st["rejected"] == 0
    assert st["resident_bytes"] == 36000 and sch.peak_in_use <= budget
    assert st["peak_bytes"] == st["resident_bytes"] + st["peak_bytes_in_flight"]
    assert sch.in_use == sch.resident  # everything in flight was released


def test_instance_whose_grid_does_not_fit_is_not_served():
    clock = FakeClock()
    insts = {0: GridInst(32, 4000, 0), 1: GridInst(32, 60000, 0)}
    sch = Scheduler(ResidentBackend(clock), insts, 50000, clock=clock)
    assert sch.unserved == {1}
    st = sch.run([Request(0, 0, 0, 0.0), Request(1, 1, 0, 0.0), Request(2, 0, 1, 0.0005)])
    assert st["requests"] == 2 and st["rejected"] == 1 and sch.rejected[0].rid == 1
    assert st["instances_unserved"] == 1


def test_hold_deadline_groups_requests():
    # arrivals every 0.2 ms for one view size on a device that takes 1 ms per
    # batch: without a hold each free slot takes what is there; with a 2 ms
    # hold (while a batch is in flight) the groups are larger, and no request
    # waits in the queue much longer than the hold plus one batch
    def run(hold):
        clock = FakeClock(tick=1e-5)
        insts = {0: Inst(32)}
        reqs = [Request(k, 0, k, 0.0002 * k) for k in range(200)]
        sch = Scheduler(FakeBackend(clock, n_streams=4), insts, 10**9, max_batch=16, clock=clock, hold_s=hold)
        st = sch.run(reqs)
        assert st["requests"] == 200
        return st, max(r.t_admit - r.t_arrival for r in sch.done)

    st0, _ = run(0.0)
    st2, wait2 = run(2e-3)
    assert st2["mean_batch"] > 2 * st0["mean_batch"]
    assert wait2 <= 2e-3 + 1.3e-3
