"""GPU tests of the update kernel that sums the next order parameter while it
holds the post-collision phase-field values (partial sums per source plane
and tile edge, merged by the next step), through the C ABI.

The pieces are added in another order than the pull sum, so the path is
compared with the FP64 oracle at the FP64 one-step tolerance over several
steps, with the pull-sum path (mode 0) at round-off, and bit for bit with
itself run to run and across block shapes (the summing kernel's tiles are
whole rows by as many rows as 512 threads (256 with FP64) allow, dividing
ny, whatever the block of the other kernels).  Cases cover tiles of one to
eight rows, walls and periodic wrap in y and z, one-tile-high lattices (the
edge sums wrap onto the same tile), the transitions that must fall back to
the pull sum (first step, a step without partial sums), the batched
form, which sums phi the same way and must give the same bits, and the
single-relaxation-time collision, whose summing update keeps the pulled flow
values in LDS instead of pulling them twice."""
import numpy as np
import pytest

import oracle
from tests.helpers import from_abi, gpu_available, rel_err, to_abi
from tests.test_gpu_parity import gpu_solver, noisy_state, random_case

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2101_06769_amd import mplb


# (n, bc): x periodic, nx a multiple of 64; y, z periodic or walls.  Tile
# rows with FP64 / FP32 arithmetic in the comments (tiles along y).
CASES = [
    ((64, 8, 6), (0, 0, 1)),     # walls in z; 4 / 8 rows (FP32: one tile)
    ((64, 8, 6), (0, 1, 1)),     # walls in y and z, corners; 4 / 8
    ((64, 6, 5), (0, 1, 0)),     # walls in y; 3 / 6 rows
    ((128, 4, 3), (0, 0, 0)),    # fully periodic, nz = 3; 2 / 4
    ((128, 2, 4), (0, 0, 1)),    # a single tile: edges wrap onto it; 2 / 2
    ((256, 3, 2), (0, 0, 0)),    # 256-wide rows, nz = 2 (both z links to one plane); 1 / 1
    ((192, 2, 3), (0, 1, 1)),    # three wavefronts per row; 1 / 2
    ((128, 8, 5), (0, 1, 1)),    # 2 / 4 rows, two tiles between walls
    ((64, 16, 4), (0, 0, 1)),    # 4 / 8 rows, two tiles, periodic y
    ((64, 1, 3), (0, 0, 1)),     # one row: both edge sums wrap onto it
    ((64, 1, 3), (0, 1, 0)),     # one row between walls in y
    ((128, 4, 1), (0, 0, 1)),    # one plane between walls in z (both z faces bounce)
    ((64, 1, 1), (0, 0, 0)),     # one row, one plane, fully periodic
]


def run(params, storage, state, fields, steps, mode, block=None):
    s = gpu_solver(params, storage, state=state, fields=fields)
    if block:
        s.set_block(*block)
    s.set_phi_partials(mode)
    s.step(steps)
    return s


@pytest.mark.parametrize("n,bc", CASES)
def test_partial_sums_match_oracle_fp64(n, bc):
    params, phi, u, p = random_case(3, n, bc, seed=sum(n) + 1)
    po, f, g = noisy_state(params, phi, u, p, seed=5, amp=0.03)
    s = run(params, "fp64", (f, g), (phi, u, p), 0, 1)
    assert s.uses_phi_partials()
    s.step(4)
    f4, g4 = oracle.step(po, f, g, 4)
    ef = rel_err(from_abi(3, s.get_populations(0)), f4)
    eg = rel_err(from_abi(3, s.get_populations(1)), g4)
    ep = rel_err(s.fields()["phi"], oracle.fields(po, f4, g4)["phi"])
    print("partial phi fp64 %s %s: f' %.2e g %.2e phi %.2e" % (n, bc, ef, eg, ep))
    assert ef < 1e-12 and eg < 1e-12 and ep < 1e-12, (ef, eg, ep)


# FP16S: a round-off difference in phi can move a stored FP16 f' code by one
# step (2^-11 of the encoded deviation), so its bar is that quantum
@pytest.mark.parametrize("storage,tol", [("fp32", 2e-5), ("fp16s", 1e-3), ("fp16s_all", 1e-3)])
@pytest.mark.parametrize("n,bc", [CASES[0], CASES[2], CASES[3], CASES[7], CASES[8],
                                  ((512, 3, 4), (0, 1, 1))])
def test_partial_sums_match_pull_sum(storage, tol, n, bc):
    params, phi, u, p = random_case(3, n, bc, seed=sum(n) + 2)
    out = []
    # rows of 512 cells: one row per 512-thread tile, FP32 arithmetic only
    summing = n[0] <= 256 or storage != "fp64"
    for mode in (1, 0):
        s = run(params, storage, None, (phi, u, p), 6, mode)
        assert s.uses_phi_partials() == (bool(mode) and summing)
        out.append((s.get_populations(0), s.get_populations(1), s.fields()["phi"]))
    for k in range(3):
        e = rel_err(out[0][k], out[1][k])
        print("partial vs pull %s %s [%d]: %.2e" % (storage, n, k, e))
        assert e < tol, (k, e)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_partial_sums_do_not_depend_on_block_shape(storage):
    params, phi, u, p = random_case(3, (128, 8, 5), (0, 1, 1), seed=71)
    out = []
    for blk in ((128, 2, 1), (64, 4, 1), (32, 2, 2), (16, 4, 1)):
        s = run(params, storage, None, (phi, u, p), 5, 1, block=blk)
        assert s.uses_phi_partials()
        out.append((blk, s.get_populations(0), s.get_populations(1), s.fields()["phi"]))
    for blk, fa, ga, pa in out[1:]:
        assert np.array_equal(fa, out[0][1]), blk
        assert np.array_equal(ga, out[0][2]), blk
        assert np.array_equal(pa, out[0][3]), blk


def test_partial_sums_deterministic_and_conserve_mass():
    params, phi, u, p = random_case(3, (128, 8, 12), (0, 0, 1), seed=31)
    outs = []
    for _ in range(2):
        s = run(params, "fp32", None, (phi, u, p), 30, 1)
        red, rc = s.reduce()
        assert rc == mplb.OK
        outs.append((s.get_populations(1), red[0]))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
    assert abs(outs[0][1] - phi.sum()) / phi.sum() < 1e-6


def test_selection_and_fallbacks():
    params, phi, u, p = random_case(3, (64, 8, 6), (0, 0, 1), seed=41)
    po, f, g = noisy_state(params, phi, u, p, seed=43, amp=0.03)
    s = gpu_solver(params, "fp64", state=(f, g), fields=(phi, u, p))
    assert s.uses_phi_partials()
    s.set_block(32, 4, 1)                   # the other kernels' block: no effect
    assert s.uses_phi_partials()
    s.set_phi_partials(0)
    assert not s.uses_phi_partials()
    with pytest.raises(mplb.MplbError):
        s.set_phi_partials(2)
    # a step without partial sums in between: the next step sums the pulled
    # populations again
    for mode, blk, steps in ((1, (64, 2, 1), 2), (0, (64, 4, 1), 1), (1, (32, 2, 2), 3),
                             (0, (64, 1, 1), 1), (1, (64, 4, 1), 1)):
        s.set_phi_partials(mode)
        s.set_block(*blk)
        s.step(steps)
    f8, g8 = oracle.step(po, f, g, 8)
    assert rel_err(from_abi(3, s.get_populations(0)), f8) < 1e-12
    assert rel_err(from_abi(3, s.get_populations(1)), g8) < 1e-12
    # layouts the path does not take
    for n, bc in (((64, 8, 6), (0, 2, 1)), ((64, 8, 6), (1, 0, 1)), ((60, 8, 6), (0, 0, 1)),
                  ((320, 2, 3), (0, 0, 1))):
        params2, phi2, u2, p2 = random_case(3, n, bc, seed=3)
        s2 = gpu_solver(params2, "fp32", fields=(phi2, u2, p2))
        assert not s2.uses_phi_partials(), (n, bc)
    s3 = gpu_solver(params, "fp16s_all", fields=(phi, u, p))
    assert s3.uses_phi_partials()  # FP16 phase-field values: sums of what the readers decode


def test_batch_run_then_solo_steps():
    # partial sums carried from solo steps into a batch run and back out
    params, phi, u, p = random_case(3, (64, 8, 6), (0, 0, 1), seed=47)
    po, f, g = noisy_state(params, phi, u, p, seed=53, amp=0.03)
    b = mplb.Batch(3, "fp64", capacity=2, max_tiles=1 << 14)
    s = mplb.Solver(params, storage="fp64", stream=b.stream)
    s.init(phi, u, p)
    s.set_populations(0, to_abi(3, f))
    s.set_populations(1, to_abi(3, g))
    s.step(2)
    assert s.uses_phi_partials()
    slot = b.attach(s, 3)
    b.step(3)
    b.detach(slot)
    s.step(2)
    f7, g7 = oracle.step(po, f, g, 7)
    assert rel_err(from_abi(3, s.get_populations(0)), f7) < 1e-12
    assert rel_err(from_abi(3, s.get_populations(1)), g7) < 1e-12


def test_first_order_equilibrium_with_partial_sums():
    params, phi, u, p = random_case(3, (64, 8, 6), (0, 1, 1), seed=59)
    params["cac_edf"] = 1
    po, f, g = noisy_state(params, phi, u, p, seed=61, amp=0.03)
    s = gpu_solver(params, "fp64", state=(f, g), fields=(phi, u, p))
    assert s.uses_phi_partials()
    s.step(3)
    f3, g3 = oracle.step(po, f, g, 3)
    assert rel_err(from_abi(3, s.get_populations(0)), f3) < 1e-12
    assert rel_err(from_abi(3, s.get_populations(1)), g3) < 1e-12


# Single relaxation time (the ablation of Sec. 4) relaxes every moment, so its
# collision needs the pulled flow values one by one, not only their moments:
# the summing update keeps them in the LDS slots of its phase-field values
# between the moment pass and the flow collision (where the flow set collides
# first), the pull-sum update pulls them again.  Several steps, so that the
# summing update runs after the first (pull-sum) step.
@pytest.mark.parametrize("n,bc", [CASES[0], CASES[2], CASES[3], CASES[7], CASES[9]])
def test_single_relaxation_time_with_partial_sums_matches_oracle_fp64(n, bc):
    params, phi, u, p = random_case(3, n, bc, seed=sum(n) + 7, collision=1)
    po, f, g = noisy_state(params, phi, u, p, seed=9, amp=0.03)
    s = run(params, "fp64", (f, g), (phi, u, p), 0, 1)
    assert s.uses_phi_partials()
    s.step(4)
    f4, g4 = oracle.step(po, f, g, 4)
    ef = rel_err(from_abi(3, s.get_populations(0)), f4)
    eg = rel_err(from_abi(3, s.get_populations(1)), g4)
    print("partial phi srt fp64 %s %s: f' %.2e g %.2e" % (n, bc, ef, eg))
    assert ef < 1e-12 and eg < 1e-12, (ef, eg)


@pytest.mark.parametrize("storage,tol", [("fp32", 2e-5), ("fp16s", 1e-3), ("fp16s_all", 1e-3)])
def test_single_relaxation_time_partial_sums_match_pull_sum(storage, tol):
    params, phi, u, p = random_case(3, (128, 8, 5), (0, 1, 1), seed=77, collision=1)
    out = []
    for mode in (1, 0):
        s = run(params, storage, None, (phi, u, p), 6, mode)
        assert s.uses_phi_partials() == bool(mode)
        out.append((s.get_populations(0), s.get_populations(1), s.fields()["phi"]))
    for k in range(3):
        e = rel_err(out[0][k], out[1][k])
        print("srt partial vs pull %s [%d]: %.2e" % (storage, k, e))
        assert e < tol, (k, e)


def nphi_batch_cases(storage_seed=0, wide=False, collision=0):
    # x-periodic domains whose update sums phi (rows of 64 / 128 / 192 cells,
    # and 512 with wide) beside ones that do not (48-wide rows), walls and
    # periodic wrap in y, z
    spec = [((64, 8, 6), (0, 0, 1)), ((128, 4, 5), (0, 0, 0)), ((48, 8, 6), (0, 1, 1)),
            ((64, 12, 4), (0, 1, 1)), ((192, 2, 3), (0, 0, 1))]
    if wide:
        spec.append(((512, 2, 3), (0, 1, 1)))
    out = []
    for k, (n, bc) in enumerate(spec):
        params, phi, u, p = random_case(3, n, bc, seed=100 + k + storage_seed, collision=collision)
        out.append((params, phi, u, p))
    return out


def batch_solver(case, storage, stream):
    params, phi, u, p = case
    s = mplb.Solver(params, storage=storage, stream=stream)
    s.init(phi, u, p)
    return s


@pytest.mark.parametrize("storage,chunk,collision", [
    ("fp32", 0, 0), ("fp32", 4, 0), ("fp64", 4, 0), ("fp16s", 4, 0), ("fp16s_all", 4, 0),
    ("fp32", 4, 1), ("fp64", 0, 1), ("fp16s", 4, 1), ("fp16s_all", 0, 1)])
def test_batch_with_phi_summing_domains_equals_alone_bitwise(storage, chunk, collision):
    wide = storage == "fp32"
    cases = nphi_batch_cases(wide=wide, collision=collision)
    steps = 7
    alone = []
    for c in cases:
        s = batch_solver(c, storage, None)
        s.step(steps)
        alone.append((s.get_populations(0), s.get_populations(1), s.fields()["phi"]))
    b = mplb.Batch(3, storage, capacity=8, max_tiles=1 << 16)
    b.set_graph_chunk(chunk)
    solvers = [batch_solver(c, storage, b.stream) for c in cases]
    want = [True, True, False, True, True] + ([True] if wide else [])
    assert [s.uses_phi_partials() for s in solvers] == want
    for s in solvers:
        b.attach(s, steps)
    b.step(steps + 3)
    for k, (s, want) in enumerate(zip(solvers, alone)):
        got = (s.get_populations(0), s.get_populations(1), s.fields()["phi"])
        for j in range(3):
            assert np.array_equal(got[j], want[j]), (storage, k, j)


def test_batch_windows_and_solo_steps_around_them_equal_alone():
    # solo steps (leaving partial sums), a batch window opened mid-batch, solo
    # steps after it: the same bits as one solo run of the same length
    cases = nphi_batch_cases(storage_seed=7)
    plan = [(2, 0, 3, 2), (0, 1, 4, 1), (1, 2, 2, 3), (3, 0, 5, 0), (0, 3, 3, 2)]
    alone = []
    for c, (pre, _, n, post) in zip(cases, plan):
        s = batch_solver(c, "fp32", None)
        s.step(pre + n + post)
        alone.append((s.get_populations(0), s.get_populations(1)))
    b = mplb.Batch(3, "fp32", capacity=8, max_tiles=1 << 16)
    b.set_graph_chunk(2)
    solvers = [batch_solver(c, "fp32", b.stream) for c in cases]
    for s, (pre, _, _, _) in zip(solvers, plan):
        s.step(pre)
    slots = {}
    for t in range(8):
        for i, (_, at, n, _) in enumerate(plan):
            if t == at:
                slots[i] = b.attach(solvers[i], n)
        b.step(1)
    for i, sl in slots.items():
        assert b.remaining(sl) == 0
        b.detach(sl)
    for i, (s, (pre, _, n, post)) in enumerate(zip(solvers, plan)):
        s.step(post)
        assert s.steps_done() == pre + n + post
        fa, ga = s.get_populations(0), s.get_populations(1)
        assert np.array_equal(fa, alone[i][0]) and np.array_equal(ga, alone[i][1]), i
