"""One step of the HIP path against the FP64 oracle at the full sizes the
benchmark runs, in the launch configuration bench.py times, checked at sampled
cells (the oracle's step at chosen cells only, pinned to its full step in
test_oracle_sampled_reduce):

* the 3-D Rayleigh-Taylor workload, 128 x 128 x 512 (Sec. 3.3 shape; At 0.5,
  Re 1000, W 5), ten steps in, with the update that sums the next phi: FP64,
  FP16S and FP16S_ALL (FP32 is in test_gpu_parity);
* the largest served lattice, a 1024 x 1024 2-D Rayleigh-Taylor domain
  (Sec. 3.2 shape), FP32 and FP64;
* the droplet impact on a thin sheet at its full size, 512 x 512 x 256
  (Sec. 3.4; density ratio 1000, viscosity ratio 15, We 8000, Re 1000,
  D = 64), in FP32 and FP16S, ten steps in (about 60 GB of host memory for
  the decoded states);
* a 3-D Rayleigh-Taylor lattice past the 32-bit population offsets,
  512 x 512 x 304 (27 x 79.7M > 2^31 elements per population array), which
  takes the per-lane addressing with 64-bit plane offsets and the phi pass
  instead of the row form and the partial sums, FP32, two steps in.

The oracle starts from the GPU's own decoded state at the sampled cells' level.
The samples are seeded random cells plus both wall layers.  FP64 and FP32 are
held to the one-step bars (1e-12, 2e-6 relative); the FP16 formats are
compared in the stored representation as in test_gpu_fp16 (one FP16 ulp of
the code plus an FP32 term plus one FP16 step of a reference), and their FP32
rest values against the oracle's within the FP16 quanta of the moving values
the cell wrote (the rest value is their remainder; the exact remainder check,
which needs every reader of a cell, runs on the small lattices of
test_gpu_fp16).
"""
import numpy as np
import pytest

import oracle
from paper_2101_06769_amd import inputs
from tests.helpers import from_abi, gpu_available, rel_err, to_abi
from tests.test_gpu_fp16 import (check_q, flow_q, phase_q, refs16, source_at, ulp16,
                                 weights_abi)

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2101_06769_amd import mplb

TOL1 = {"fp64": 1e-12, "fp32": 2e-6}


def sample(n, count, seed):
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    layer = nx * ny if nz > 1 else nx
    last = nx * ny * nz - layer
    return np.concatenate([rng.integers(0, nx * ny * nz, count),
                           rng.integers(0, layer, count // 6),           # first wall layer
                           last + rng.integers(0, layer, count // 6)])  # last wall layer


def run(case, storage, warm):
    """GPU state (decoded, oracle order) after `warm` steps and after one more."""
    dim = case.params["dim"]
    s = mplb.Solver(case.params, storage=storage)
    s.init(case.phi, case.u, case.p)
    s.step(warm)
    f = from_abi(dim, s.get_populations(0))
    g = from_abi(dim, s.get_populations(1))
    s.step(1)
    return s, f, g, s.get_populations(0), s.get_populations(1)


def full_rti3d():
    return inputs.rti3d()


def full_rti2d():
    return inputs.rti2d(nx=1024, ny=1024, amp=0.05 * 1024)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_largest_served_2d_lattice_one_step_at_sampled_cells(storage):
    case = full_rti2d()
    s, f, g, f1, g1 = run(case, storage, warm=10)
    assert s.phi_partial_rows() == 0  # 2-D: the phi pass and the update
    cells = sample(case.params["n"], 3000, seed=1)
    po = oracle.params_from_dict(case.params)
    fo, go = oracle.step_sampled(po, f, g, cells)
    fg = from_abi(2, f1).reshape(9, -1)[:, cells].T
    gg = from_abi(2, g1).reshape(9, -1)[:, cells].T
    ef, eg = rel_err(fg, fo), rel_err(gg, go)
    print("2-D 1024^2 %s one step at %d cells: f rel %.2e, g rel %.2e" % (storage, cells.size, ef, eg))
    assert ef < TOL1[storage] and eg < TOL1[storage]


def test_full_size_rti3d_fp64_one_step_at_sampled_cells():
    case = full_rti3d()
    s, f, g, f1, g1 = run(case, "fp64", warm=10)
    assert s.phi_partial_rows() > 0  # the benchmark's step form
    cells = sample(case.params["n"], 1500, seed=2)
    po = oracle.params_from_dict(case.params)
    fo, go = oracle.step_sampled(po, f, g, cells)
    fg = from_abi(3, f1).reshape(27, -1)[:, cells].T
    gg = from_abi(3, g1).reshape(27, -1)[:, cells].T
    ef, eg = rel_err(fg, fo), rel_err(gg, go)
    print("3-D 128x128x512 fp64 one step at %d cells: f rel %.2e, g rel %.2e" % (cells.size, ef, eg))
    assert ef < 1e-12 and eg < 1e-12


def check_fp16_sampled(case, storage, f, g, got_f, got_g, cells, label):
    """FP16 stored representation at sampled cells: f, g the decoded state
    (oracle order) the step started from; got_f, got_g the GPU's decoded
    populations after it at the cells ([Q][m], library order)."""
    dim, params = 3, case.params
    n, bc = params["n"], params["bc"]
    po = oracle.params_from_dict(params)
    fo_c, go_c = oracle.step_sampled(po, f, g, cells)
    fo = to_abi(dim, fo_c.T)  # [Q][m], library order
    go = to_abi(dim, go_c.T)
    # the writers' references: fp16 of p* and phi of the level the step started from
    fl = oracle.fields(po, f, g)
    refs = refs16(params, fl["phi"], fl["p"])
    nx, ny = n[0], n[1]
    x, y, z = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    src = source_at(dim, n, bc, x, y, z)
    w = weights_abi(dim).reshape(-1, 1)
    Q = 27
    # flow set: codes against the writers' references
    qo, dref = flow_q(dim, fo, refs, src)
    qg, _ = flow_q(dim, got_f, refs, src)
    s_src = refs[2].ravel()[src]
    check_q(qg, qo, 4e-6 * np.abs(fo).max() / (w * s_src) + dref)
    # FP32 rest value: the remainder over the moving values the cell wrote,
    # each off the exact value by at most half an FP16 step of its code times
    # w s (the reference P cancels), plus FP32 round-off of the sums
    s_me = refs[2].ravel()[cells]
    qmax = np.abs(qo).max()
    bar = (1 - w[Q // 2, 0]) * s_me * ulp16(qmax) + 1e-5 * np.abs(fo).max()
    drest = np.abs(got_f[Q // 2] - fo[Q // 2])
    print("%s %s flow: max code diff %.3g, rest diff %.2e (bar %.2e)" %
          (label, storage, np.abs(qg - qo).max(), drest.max(), bar.max()))
    assert np.all(drest <= bar)
    if storage == "fp16s":
        assert rel_err(got_g, go) < 2e-6
    else:
        F = refs[1].ravel()[cells]  # the readers are the sampled cells
        qo, dref = phase_q(dim, go, F)
        qg, _ = phase_q(dim, got_g, F)
        check_q(qg, qo, 4e-6 * (np.abs(qo).max() + 1.0) + dref)
        barg = (1 - w[Q // 2, 0]) * ulp16(np.abs(qo).max()) + 1e-5
        dg = np.abs(got_g[Q // 2] - go[Q // 2])
        print("  phase: max code diff %.3g, rest diff %.2e (bar %.2e)" %
              (np.abs(qg - qo).max(), dg.max(), barg))
        assert dg.max() <= barg


@pytest.mark.parametrize("storage", ["fp16s", "fp16s_all"])
def test_full_size_rti3d_fp16_one_step_at_sampled_cells(storage):
    case = full_rti3d()
    s, f, g, f1, g1 = run(case, storage, warm=10)
    assert s.phi_partial_rows() > 0
    cells = sample(case.params["n"], 1500, seed=3)
    got_f = f1.reshape(27, -1)[:, cells]
    got_g = g1.reshape(27, -1)[:, cells]
    del f1, g1
    check_fp16_sampled(case, storage, f, g, got_f, got_g, cells, "3-D 128x128x512")


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_full_size_splash_one_step_at_sampled_cells(storage):
    # the benchmark's droplet impact at full size; the populations are read
    # back one set at a time and only the sampled columns of the stepped
    # state are kept, to bound host memory
    case = inputs.splash3d()
    s = mplb.Solver(case.params, storage=storage)
    s.init(case.phi, case.u, case.p)
    s.step(10)
    f = from_abi(3, s.get_populations(0))
    g = from_abi(3, s.get_populations(1))
    s.step(1)
    cells = sample(case.params["n"], 1500, seed=4)
    got_f = s.get_populations(0).reshape(27, -1)[:, cells]
    got_g = s.get_populations(1).reshape(27, -1)[:, cells]
    del s
    if storage == "fp32":
        po = oracle.params_from_dict(case.params)
        fo, go = oracle.step_sampled(po, f, g, cells)
        ef = rel_err(from_abi(3, got_f).T, fo)
        eg = rel_err(from_abi(3, got_g).T, go)
        print("3-D splash 512x512x256 fp32 one step at %d cells: f rel %.2e, g rel %.2e" %
              (cells.size, ef, eg))
        assert ef < 2e-6 and eg < 2e-6
    else:
        check_fp16_sampled(case, storage, f, g, got_f, got_g, cells, "3-D splash 512x512x256")


def test_lattice_past_32bit_population_offsets_one_step_at_sampled_cells():
    # 512 x 512 x 304: 79.7M cells, 27 x 79.7M population elements per array,
    # past 2^31, so the kernels index planes with 64-bit offsets (per-lane
    # form); host memory for the decoded states about 70 GB at the peak
    case = inputs.rti3d(nx=512, ny=512, nz=304, amp=0.05 * 512)
    n = case.params["n"]
    assert 27 * n[0] * n[1] * n[2] > 2 ** 31
    s = mplb.Solver(case.params, storage="fp32")
    s.init(case.phi, case.u, case.p)
    assert s.phi_partial_rows() == 0  # past the 32-bit offsets: the phi pass
    s.step(2)
    f = from_abi(3, s.get_populations(0))
    g = from_abi(3, s.get_populations(1))
    s.step(1)
    cells = sample(n, 1500, seed=5)
    got_f = s.get_populations(0).reshape(27, -1)[:, cells]
    got_g = s.get_populations(1).reshape(27, -1)[:, cells]
    del s
    po = oracle.params_from_dict(case.params)
    fo, go = oracle.step_sampled(po, f, g, cells)
    ef = rel_err(from_abi(3, got_f).T, fo)
    eg = rel_err(from_abi(3, got_g).T, go)
    print("3-D 512x512x304 fp32 one step at %d cells: f rel %.2e, g rel %.2e" % (cells.size, ef, eg))
    assert ef < 2e-6 and eg < 2e-6
