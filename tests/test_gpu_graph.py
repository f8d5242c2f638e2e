"""mplb_step replays runs of steady-state steps as a captured graph.  Each
replay must give the bits of the same steps launched one by one: compared
after every replay, with host reads, synchronisation and other device work
between the replays, across a change of launch block and of step form (which
recapture), and across a checkpoint load that changes the level parity."""
import numpy as np
import pytest

from paper_2101_06769_amd import inputs
from tests.helpers import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    from paper_2101_06769_amd import mplb

CHUNK = 16  # steps per graph launch of mplb_step


def _state(s):
    return s.get_populations(0), s.get_populations(1)


def _pair(case, storage, edf=0):
    params = dict(case.params, cac_edf=edf)
    a = mplb.Solver(params, storage=storage)
    b = mplb.Solver(params, storage=storage)
    for s in (a, b):
        s.init(case.phi, case.u, case.p)
    return a, b


def _cases():
    return {
        "rti3d": inputs.rti3d(nx=64, ny=8, nz=24, amp=2.0),       # the phi-summing update
        "drop2d": inputs.static_droplet(dim=2, n=(48, 40, 1), R=10.0, sigma=1e-3, rho_ratio=1000.0),
    }


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16s", "fp16s_all"])
@pytest.mark.parametrize("kind,edf", [("rti3d", 0), ("rti3d", 1), ("drop2d", 0)])
def test_graph_replays_equal_steps_one_by_one(storage, kind, edf):
    case = _cases()[kind]
    a, b = _pair(case, storage, edf)
    a.step(3)  # the first steps run directly (no history, no partial sums yet)
    for _ in range(3):
        b.step(1)
    for rep in range(4):
        a.step(CHUNK)              # one graph launch
        for _ in range(CHUNK):     # the same steps launched one by one
            b.step(1)
        # eager work and synchronisation between the replays
        scratch = torch.ones(1 << 20, device="cuda") * float(rep)
        torch.cuda.synchronize()
        assert float(scratch.sum()) == float(rep) * (1 << 20)
        fa, ga = _state(a)
        fb, gb = _state(b)
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), (storage, kind, edf, rep)
        assert a.steps_done() == b.steps_done()


def test_graph_follows_block_and_step_form_changes_and_loads():
    case = _cases()["rti3d"]
    a, b = _pair(case, "fp32")
    a.step(1 + CHUNK)
    for _ in range(1 + CHUNK):
        b.step(1)
    # another launch block: a new graph
    a.set_block(64, 2, 2)
    b.set_block(64, 2, 2)
    a.step(CHUNK)
    for _ in range(CHUNK):
        b.step(1)
    assert all(np.array_equal(x, y) for x, y in zip(_state(a), _state(b)))
    # the phi pass instead of the partial sums: another step form
    a.set_phi_partials(0)
    b.set_phi_partials(0)
    a.step(1 + CHUNK)
    for _ in range(1 + CHUNK):
        b.step(1)
    assert all(np.array_equal(x, y) for x, y in zip(_state(a), _state(b)))
    # a load at the other level parity
    blob = b.save()
    b.step(1)
    a.load(b.save())
    a.step(CHUNK)
    for _ in range(CHUNK):
        b.step(1)
    assert all(np.array_equal(x, y) for x, y in zip(_state(a), _state(b)))
    a.load(blob)
    c = mplb.Solver(case.params, storage="fp32")
    c.load(blob)
    a.step(CHUNK)
    for _ in range(CHUNK):
        c.step(1)
    assert all(np.array_equal(x, y) for x, y in zip(_state(a), _state(c)))
