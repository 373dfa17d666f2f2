"""Host logic of the continuous-batching server (no GPU): a request larger
than the whole batch is rejected at admission instead of waiting forever and
holding up the requests behind it."""
from paper_2208_13769_amd import serve


class _FakeBatch:
    """Stands in for a batch whose arena holds plates of at most `limit` sites
    per side; plates finish after one chunk."""

    def __init__(self, limit):
        self.limit = limit
        self.live = {}
        self.next = 0

    def fits_empty(self, nx, ny):
        return max(nx, ny) <= self.limit

    def add(self, spec, u0, v0, nsteps):
        if not self.fits_empty(spec.nx, spec.ny) or self.live:
            return None
        self.next += 1
        self.live[self.next] = nsteps
        return self.next

    def step(self, n):
        for k in self.live:
            self.live[k] = 0

    def synchronize(self):
        pass

    def query(self, slot):
        return (1, self.live[slot], False)

    def read(self, slot):
        return None

    def retire(self, slot):
        del self.live[slot]


def test_requests_larger_than_the_batch_are_rejected():
    reqs = serve.make_requests(6, 11, n_median=64, steps_max=600)
    for r in reqs:
        r.arrival = 0.0
    limit = sorted(r.n for r in reqs)[2]  # the three largest cannot fit
    srv = serve.BatchServer(0, batch=_FakeBatch(limit))
    summ, finish, _ = srv.run(reqs)
    too_big = {r.rid for r in reqs if r.n > limit}
    assert set(summ["rejected_ids"]) == too_big and summ["rejected"] == len(too_big)
    assert set(finish) == {r.rid for r in reqs} - too_big
    assert summ["p99_s"] >= summ["p50_s"] >= 0.0
