"""Server logic on a host-only backend with a simulated clock: every request
runs all its steps, none starts before it arrives, admission respects the
memory cap and arrival order, and latency bookkeeping is consistent."""
from paper_1103_3373_amd.serve import HostBackend, Request, Server, footprint_bytes
from paper_1103_3373_amd import workloads as W


def _stream(n=60, rate=200.0, steps=5, seed=1):
    reqs = W.request_stream(n_requests=n, rate=rate, seed=seed)
    return [Request(r["id"], r["arrival"], r["n"], r["scheme"], r["riemann"], r["ic"], r["seed"], steps)
            for r in reqs]


def test_all_requests_complete_with_their_steps():
    be = HostBackend()
    srv = Server(be, mem_cap=200e9, clock=be.clock)
    reqs = _stream()
    for r in reqs:
        srv.submit(r)
    srv.run()
    assert len(srv.done) == len(reqs)
    for r in reqs:
        sim = srv.done[r.id]
        assert sim.step == r.steps and len(sim.latencies) == r.steps
        assert sim.admitted >= r.arrival - 1e-12
        assert all(l > 0 for l in sim.latencies)
    assert srv.used == 0
    rep = srv.report()
    assert rep["requests"] == len(reqs)
    assert rep["cell_updates"] == sum(r.n ** 3 * r.steps for r in reqs)
    assert rep["p99_step_latency_ms"] >= rep["p50_step_latency_ms"] > 0


def test_memory_cap_backpressure_and_fifo_admission():
    be = HostBackend(s_per_cell=1e-9)
    reqs = _stream(n=40, rate=1e4, steps=3)
    cap = max(footprint_bytes(r) for r in reqs) * 2  # at most a couple at a time
    srv = Server(be, mem_cap=cap, clock=be.clock)
    for r in reqs:
        srv.submit(r)
    peak = []
    orig = srv._admit

    def spy(now):
        out = orig(now)
        peak.append(srv.used)
        return out

    srv._admit = spy
    srv.run()
    assert len(srv.done) == len(reqs)
    assert max(peak) <= cap
    order = sorted(srv.done.values(), key=lambda s: s.admitted)
    arrivals = [s.req.arrival for s in order]
    assert arrivals == sorted(arrivals)  # admitted in arrival order
    assert srv.report()["mean_admission_wait_ms"] > 0  # requests had to wait


def test_requests_join_while_others_run():
    """Continuous batching: a request arriving mid-run is stepped together
    with the ones already active (ticks contain several simulations)."""
    be = HostBackend(s_per_cell=1e-9, s_fixed=1e-3)
    reqs = [Request(0, 0.0, 32, 2, 1, "sod", 0, 20), Request(1, 0.005, 32, 0, 0, "blast", 0, 20)]
    srv = Server(be, clock=be.clock)
    for r in reqs:
        srv.submit(r)
    sizes = []
    orig = be.tick

    def spy(handles):
        sizes.append(len(handles))
        return orig(handles)

    be.tick = spy
    srv.run()
    assert max(sizes) == 2 and sizes[0] == 1
    assert srv.done[1].admitted < srv.done[0].finished


def test_oversized_request_rejected():
    srv = Server(HostBackend(), mem_cap=1e6)
    try:
        srv.submit(Request(0, 0.0, 128, 2, 1, "sod", 0))
    except ValueError:
        return
    raise AssertionError("oversized request accepted")
