"""GPU serving: each request's final state is bit-identical alone and inside
a mixed continuous-batching stream (different sizes, schemes, solvers and
initial conditions sharing batched launches)."""
import numpy as np
import pytest

from paper_1103_3373_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_results_same_alone_and_in_mix():
    from paper_1103_3373_amd.serve import GpuBackend, Request, Server
    reqs = [Request(i, 0.002 * i, n, s, rs, ic, i % 3, 6)
            for i, (n, s, rs, ic) in enumerate([(32, 2, 1, "sod"), (64, 0, 0, "blast"), (32, 1, 1, "lognormal"),
                                                 (32, 2, 0, "blast"), (64, 1, 0, "sod"), (32, 0, 1, "lognormal"),
                                                 (32, 2, 1, "lognormal"), (64, 2, 1, "sod")])]
    cache = {}
    be = GpuBackend(ic_cache=cache, keep_results=True)
    srv = Server(be)
    for r in reqs:
        srv.submit(r)
    srv.run()
    assert len(srv.done) == len(reqs)
    ticks = [len(s.latencies) for s in srv.done.values()]
    assert all(t == 6 for t in ticks)
    for r in reqs:
        alone_be = GpuBackend(ic_cache=cache, keep_results=True)
        alone = Server(alone_be)
        alone.submit(Request(r.id, 0.0, r.n, r.scheme, r.riemann, r.ic, r.seed, r.steps))
        alone.run()
        a = be.final_state(r.id).numpy()
        b = alone_be.final_state(r.id).numpy()
        assert np.isfinite(a).all()
        np.testing.assert_array_equal(a, b)
        assert not np.array_equal(a, cache[(r.ic, r.n, r.seed)].numpy())  # it did evolve
    rep = srv.report()
    assert rep["p50_step_latency_ms"] > 0 and rep["cell_updates"] == sum(r.n ** 3 * 6 for r in reqs)
