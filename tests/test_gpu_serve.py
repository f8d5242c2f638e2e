"""GPU tests of the serving loop: requests admitted over time by a device-
memory budget, advanced together in batched launches; every result must be
bitwise the result of the same request run alone, and the budget must hold."""
import numpy as np
import pytest

from paper_2101_06769_amd import inputs, serve
from tests.helpers import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2101_06769_amd import mplb


def small_specs(count=10, seed=5):
    return inputs.serving_spec(seed=seed, count=count, rate=40.0, edge_range=(24, 72),
                               steps_range=(20, 160), rho_ratio_range=(3.0, 30.0))


def alone(spec, storage="fp32"):
    case = inputs.serving_case(spec)
    s = mplb.Solver(case.params, storage=storage)
    s.init(case.phi, case.u, case.p)
    s.step(spec["steps"])
    return s.fields()


def test_served_results_equal_alone_and_budget_holds():
    specs = small_specs()
    sizes = sorted(serve._arena_bytes(inputs.serving_case(s), "fp32") for s in specs)
    budget = sum(sizes[-3:])  # at most about three requests resident: forces queueing
    events = []
    # every request visible at once: admission is limited by the budget alone,
    # so later requests join while earlier ones are still running
    res, st = serve.serve_batched(specs, hbm_budget=budget, capacity=8, quantum=16, chunk=4,
                                  keep_fields=True, realtime=False,
                                  on_event=lambda *e: events.append(e))
    assert st["peak_bytes"] <= budget
    assert st["peak_active"] >= 2  # work overlapped on the device
    assert len(res) == len(specs) and all(r.status == mplb.OK for r in res)
    # a request admitted while another was running: continuous batching
    admits = [e for e in events if e[0] == "admit" and e[2] > 1]
    assert admits
    for spec, r in zip(specs, res):
        assert r.id == spec["id"] and r.latency > 0
        want = alone(spec)
        for k in ("phi", "u", "p"):
            assert np.array_equal(r.fields[k], want[k]), (spec["id"], k)


def test_fifo_baseline_matches_and_oversized_requests_are_rejected():
    specs = small_specs(count=4, seed=8)
    res = serve.serve_fifo(specs, keep_fields=True, realtime=False)
    for spec, r in zip(specs, res):
        want = alone(spec)
        assert np.array_equal(r.fields["phi"], want["phi"])
    # a budget smaller than one request: it is rejected, the others still run
    big = max(specs, key=lambda s: s["edge"])
    budget = serve._arena_bytes(inputs.serving_case(big), "fp32") - 1
    res, st = serve.serve_batched(specs, hbm_budget=budget, capacity=4, realtime=False)
    rej = [r for r in res if r.status == mplb.ENOMEM]
    assert big["id"] in st["rejected"] and len(rej) >= 1
    assert all(r.status == mplb.OK for r in res if r.id not in st["rejected"])
