"""GPU tests of checkpoint / resume (mplb_save, mplb_load) and of the batch's
per-domain health flags (mplb_batch_status).

Resume: N steps must equal N/2 steps, a save, a load into a fresh solver on
its own arena, and N/2 more steps, bit for bit, in every storage format, for
the update that sums the next phi (its partial sums are part of the state)
and for the first-order phase-field equilibrium (its (phi u) history is).

Health: a domain whose state holds a non-finite value is flagged by the
batch's phi stage and retired by mplb_batch_status; the other domains of
the batch keep their bits (each equals the same domain stepped alone).
"""
import numpy as np
import pytest

from paper_2101_06769_amd import inputs, serve
from tests.helpers import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2101_06769_amd import mplb


def _state(s):
    return s.get_populations(0), s.get_populations(1)


def _case(kind):
    if kind == "rti3d":   # the phi-summing update (rows of 64 cells)
        return inputs.rti3d(nx=64, ny=8, nz=24, amp=2.0)
    if kind == "drop2d":  # 2-D, density ratio 1000, surface tension
        return inputs.static_droplet(dim=2, n=(48, 40, 1), R=10.0, sigma=1e-3, rho_ratio=1000.0)
    raise ValueError(kind)


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16s", "fp16s_all"])
@pytest.mark.parametrize("kind,edf", [("rti3d", 0), ("rti3d", 1), ("drop2d", 0), ("drop2d", 1)])
def test_save_half_load_half_equals_uninterrupted_bitwise(storage, kind, edf):
    case = _case(kind)
    params = dict(case.params, cac_edf=edf)
    n = 10
    ref = mplb.Solver(params, storage=storage)
    ref.init(case.phi, case.u, case.p)
    ref.step(n)
    a = mplb.Solver(params, storage=storage)
    a.init(case.phi, case.u, case.p)
    a.step(n // 2)
    blob = a.save()
    del a
    b = mplb.Solver(params, storage=storage)  # a fresh arena
    b.load(blob)
    assert b.steps_done() == n // 2
    b.step(n - n // 2)
    fa, ga = _state(ref)
    fb, gb = _state(b)
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb), (storage, kind, edf)
    if kind == "rti3d" and storage in ("fp32", "fp64", "fp16s"):
        assert b.uses_phi_partials()  # the partial sums travelled in the blob


def test_load_rejects_other_parameters_and_truncated_blobs():
    case = _case("rti3d")
    s = mplb.Solver(case.params, storage="fp32")
    with pytest.raises(mplb.MplbError) as e:
        s.save()  # nothing to save before init
    assert e.value.code == mplb.ESTATE
    s.init(case.phi, case.u, case.p)
    s.step(3)
    blob = s.save()
    other = mplb.Solver(dict(case.params, sigma=case.params["sigma"] + 1e-4), storage="fp32")
    with pytest.raises(mplb.MplbError) as e:
        other.load(blob)
    assert e.value.code == mplb.EINVAL
    fresh = mplb.Solver(case.params, storage="fp32")
    with pytest.raises(mplb.MplbError) as e:
        fresh.load(blob[:-1])
    assert e.value.code == mplb.EINVAL
    with pytest.raises(mplb.MplbError) as e:
        fresh.load(b"x" * len(blob))
    assert e.value.code == mplb.EINVAL
    # a header whose launch block is corrupt (the saved block shape, three
    # int32 after magic, format, region count, parameter hash, step count and
    # five int32 of bookkeeping: bytes 52..63) is refused, not launched
    bad = bytearray(blob)
    bad[52:56] = (0).to_bytes(4, "little")
    with pytest.raises(mplb.MplbError) as e:
        fresh.load(bytes(bad))
    assert e.value.code == mplb.EINVAL
    fresh.load(blob)  # the intact blob still loads


def test_attached_solver_refuses_solo_calls():
    case = _case("rti3d")
    b = mplb.Batch(3, "fp32", capacity=2, max_tiles=1 << 12)
    s = mplb.Solver(case.params, storage="fp32", stream=b.stream)
    s.init(case.phi, case.u, case.p)
    blob = s.save()
    b.attach(s, 5)
    for call in (lambda: s.step(1), lambda: s.step_timed(1), lambda: s.tune_block(1),
                 lambda: s.init(case.phi, case.u, case.p), lambda: s.load(blob),
                 lambda: s.set_populations(0, s.get_populations(0)),
                 lambda: s.set_phi_partials(0)):
        with pytest.raises(mplb.MplbError) as e:
            call()
        assert e.value.code == mplb.ESTATE


def _nan_case(case):
    phi = case.phi.copy()
    phi.reshape(-1)[phi.size // 2] = np.nan
    return inputs.Case(case.name, dict(case.params), phi, case.u, case.p, case.steps,
                       dict(case.meta))


@pytest.mark.parametrize("chunk", [0, 4])
def test_batch_flags_and_retires_a_nonfinite_domain_others_keep_their_bits(chunk):
    cases = inputs.batch_rti3d(count=4, seed=11, edges=(8, 12, 16), steps=30)
    cases[1] = _nan_case(cases[1])
    steps = 16
    alone = {}
    for k, c in enumerate(cases):
        if k == 1:
            continue
        s = mplb.Solver(c.params, storage="fp32")
        s.init(c.phi, c.u, c.p)
        s.step(steps)
        alone[k] = _state(s)
    b = mplb.Batch(3, "fp32", capacity=4, max_tiles=1 << 14)
    b.set_graph_chunk(chunk)
    solvers, slots = [], []
    for c in cases:
        s = mplb.Solver(c.params, storage="fp32", stream=b.stream)
        s.init(c.phi, c.u, c.p)
        solvers.append(s)
        slots.append(b.attach(s, steps))
    b.step(4)
    st = b.status()
    assert st[slots[1]] == mplb.EUNSTABLE
    assert all(st[slots[k]] == mplb.OK for k in (0, 2, 3))
    assert b.remaining(slots[1]) == 0  # retired: its window is closed
    done_bad = solvers[1].steps_done()
    b.step(steps)  # the others finish; the retired one takes no step
    assert solvers[1].steps_done() == done_bad
    b.detach(slots[1])
    st = b.status()
    assert slots[1] not in st
    for k, s in enumerate(solvers):
        if k == 1:
            continue
        fb, gb = _state(s)
        assert np.array_equal(alone[k][0], fb) and np.array_equal(alone[k][1], gb), k
    # a new solver in the retired slot starts with a clear flag
    c = cases[0]
    s = mplb.Solver(c.params, storage="fp32", stream=b.stream)
    s.init(c.phi, c.u, c.p)
    sl = b.attach(s, 2)
    b.step(2)
    assert b.status()[sl] == mplb.OK


def test_serving_retires_an_unstable_request_and_serves_the_rest_bitwise():
    specs = inputs.serving_spec(seed=5, count=5, rate=40.0, edge_range=(24, 64),
                                steps_range=(40, 120), rho_ratio_range=(3.0, 30.0))
    bad = dict(specs[2])
    bad["case"] = _nan_case(inputs.serving_case(bad))
    specs[2] = bad
    events = []
    res, st = serve.serve_batched(specs, hbm_budget=1 << 30, capacity=8, quantum=16, chunk=4,
                                  keep_fields=True, realtime=False,
                                  on_event=lambda *e: events.append(e))
    by_id = {r.id: r for r in res}
    r_bad = by_id[bad["id"]]
    assert r_bad.status == mplb.EUNSTABLE and r_bad.fields is None
    # retired after the quantum that flagged it, before its own last step
    # and before any other request finished
    kinds = [(e[0], e[1]) for e in events if e[0] != "admit"]
    assert kinds[0] == ("unstable", bad["id"])
    for spec in specs:
        if spec["id"] == bad["id"]:
            continue
        r = by_id[spec["id"]]
        assert r.status == mplb.OK
        case = inputs.serving_case(spec)
        s = mplb.Solver(case.params, storage="fp32")
        s.init(case.phi, case.u, case.p)
        s.step(spec["steps"])
        want = s.fields()
        for k in ("phi", "u", "p"):
            assert np.array_equal(r.fields[k], want[k]), (spec["id"], k)
