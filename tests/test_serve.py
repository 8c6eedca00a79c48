"""Host logic of the continuous-batching request loop, on a fake backend
(no GPU): admission limits, every energy solved exactly once and routed to
its request, requests joining running batches, time limits, rejection."""
import collections

import numpy as np

from paper_1903_00548_amd import serve

Dev = collections.namedtuple("Dev", "N m uniform tag")


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Deterministic stand-in: T(E) = 1000 tag + E, ldos = tag; each solve
    advances the clock by 1 ms per energy."""

    def __init__(self, clock, server_ref):
        self.clock = clock
        self.server = server_ref
        self.calls = []
        self.open_handles = 0
        self.max_open = 0

    def open(self, dev):
        self.open_handles += 1
        self.max_open = max(self.max_open, self.open_handles)
        return {"dev": dev, "closed": False}

    def solve(self, handles, grids):
        assert all(not h["closed"] for h in handles)
        srv = self.server[0]
        assert srv.used <= srv.hbm_budget and len(handles) <= srv.max_active
        self.calls.append([h["dev"].tag for h in handles])
        self.clock.t += 1e-3 * sum(len(g) for g in grids)
        Ts = [1000.0 * h["dev"].tag + np.asarray(g) for h, g in zip(handles, grids)]
        Ls = [np.full((len(g), 2, h["dev"].N), float(h["dev"].tag)) for h, g in zip(handles, grids)]
        return Ts, Ls, 0

    def close(self, h):
        assert not h["closed"]
        h["closed"] = True
        self.open_handles -= 1


def _server(**kw):
    clock = Clock()
    ref = [None]
    be = FakeBackend(clock, ref)
    srv = serve.Server(be, clock=clock, sleep=clock.sleep, **kw)
    ref[0] = srv
    return srv, be, clock


def _requests(n, seed=0, nE=(5, 40), spacing=0.01):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        d = Dev(N=int(rng.integers(2, 9)), m=int(rng.choice([8, 32, 100])), uniform=bool(k % 2), tag=k)
        E = np.sort(rng.uniform(-1, 1, int(rng.integers(*nE))))
        out.append(serve.Request(rid=k, t_arrival=k * spacing, device=d, E=E))
    return out


def test_every_energy_solved_once_and_routed():
    srv, be, _ = _server(max_active=3, energies_per_step=7)
    reqs = _requests(12)
    st = srv.run(reqs)
    assert st["completed"] == 12 and st["unfinished"] == 0 and st["rejected"] == 0
    for r in reqs:
        assert np.array_equal(r.T, 1000.0 * r.device.tag + r.E)
        assert np.all(r.ldos == r.device.tag)
        assert r.t_done >= r.t_admit >= r.t_arrival
    assert st["energies_solved"] == sum(len(r.E) for r in reqs)
    assert be.open_handles == 0 and srv.used == 0
    assert be.max_open <= 3


def test_requests_join_running_batches():
    srv, be, _ = _server(max_active=8, energies_per_step=4)
    reqs = _requests(6, nE=(30, 31), spacing=0.005)
    srv.run(reqs)
    # a request that arrived while another was being solved shares launches with it
    assert any(len(c) >= 2 for c in be.calls)
    first = {t: min(i for i, c in enumerate(be.calls) if t in c) for t in range(6)}
    assert first[5] > 0 and any(0 in c and 5 in c for c in be.calls)


def test_hbm_budget_limits_admission():
    reqs = _requests(10, nE=(20, 21))
    fps = [serve.request_footprint(r.device.N, r.device.m, len(r.E), r.device.uniform, 4) for r in reqs]
    budget = 2 * max(fps)
    srv, be, _ = _server(max_active=100, energies_per_step=4, hbm_budget=budget)
    st = srv.run(reqs)                       # FakeBackend asserts used <= budget at every launch
    assert st["completed"] == 10


def test_oversized_request_rejected_and_time_limit():
    reqs = _requests(4, nE=(50, 51))
    fp = serve.request_footprint(reqs[0].device.N, reqs[0].device.m, 50, reqs[0].device.uniform, 4)
    srv, be, _ = _server(max_active=4, energies_per_step=4, hbm_budget=fp - 1 if fp > 1 else 1)
    st = srv.run(reqs[:1])
    assert st["rejected"] == 1 and st["completed"] == 0
    srv, be, _ = _server(max_active=4, energies_per_step=2)
    st = srv.run(_requests(4, nE=(200, 201)), time_limit=0.05)
    assert st["unfinished"] > 0
    assert be.open_handles == 0


def test_latency_percentiles():
    srv, be, _ = _server(max_active=2, energies_per_step=10)
    st = srv.run(_requests(9, spacing=0.0))
    lat = sorted(r.latency for r in srv.done)
    assert st["p50_latency_s"] == np.percentile(lat, 50)
    assert st["p99_latency_s"] <= lat[-1] + 1e-12
