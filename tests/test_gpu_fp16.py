"""GPU parity of the FP16 storage formats against the FP64 oracle.

An FP16 set stores, per direction a and cell, a half-precision code of the
deviation of the post-collision value from a reference both the writer and
the reader of the value hold (Sec. 2.2, 2.3 values; the encoding is this
library's storage design):
* flow set: the writer's reference, f = w (P + s q), P = fp16(p*) and
  s = rho(F) cs^2 with F = fp16(phi), p* and phi those of the writing cell at
  the level it wrote;
* phase-field set (FP16S_ALL): the reader's reference, g = w (F + q),
  F = fp16(phi) of the reading cell at the writers' level;
* the rest direction of each FP16 set is stored in FP32.
The tests start the oracle from exactly the state the GPU holds (its decoded
populations), step both once and compare in the stored representation: the
GPU's code must be the oracle's value encoded the same way, to one FP16 ulp
plus an FP32 term, plus the code change one FP16 step of a reference would
cause (the GPU rounds its own FP32 p* and phi to FP16, the test the
oracle's, so a reference on a rounding boundary may differ by one step).
Over many steps the FP16 runs are held to the oracle's sensitivity when its
populations carry one FP16 rounding of the stored deviation after every
step.
"""
import numpy as np
import pytest

import oracle
from paper_2101_06769_amd import inputs
from tests.helpers import from_abi, gpu_available, rel_err, to_abi
from tests.test_gpu_parity import CONFIGS, noisy_state, random_case

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2101_06769_amd import mplb


def source_at(dim, n, bc, x, y, z):
    """src[a, ...] = flat index of the cell that wrote the value the cell at
    (x, y, z) (arrays of one shape) pulls in direction a (library order):
    x - c_a under periodic wrap, the same-side cell beyond a symmetry plane,
    the cell itself when the link leaves the domain through a wall
    (bounce-back)."""
    nx, ny, nz = n
    Q = 9 if dim == 2 else 27
    out = np.empty((Q,) + np.shape(x), dtype=np.int64)
    for a in range(Q):
        c = (a % 3 - 1, (a // 3) % 3 - 1, (a // 9 - 1) if dim == 3 else 0)
        coords, wall = [], np.zeros(np.shape(x), bool)
        for comp, xi, ni, bci in zip(c, (x, y, z), (nx, ny, nz), bc):
            s = xi - comp
            outside = (s < 0) | (s >= ni)
            if bci == 0:
                s = np.mod(s, ni)
            elif bci == 1:
                wall |= outside
                s = np.where(outside, xi, s)
            else:
                s = np.where(outside, xi, s)
            coords.append(s)
        sx, sy, sz = coords
        src = (sz * ny + sy) * nx + sx
        me = (z * ny + y) * nx + x
        out[a] = np.where(wall, me, src)
    return out


def source_cells(dim, n, bc):
    """source_at for every cell, shaped [Q][nz][ny][nx]."""
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return source_at(dim, n, bc, x, y, z)


def ulp16(v):
    """Spacing of FP16 numbers at |v| (subnormal spacing 2^-24 below 2^-14)."""
    a = np.maximum(np.abs(v), 2.0 ** -14)
    return 2.0 ** (np.floor(np.log2(a)) - 10)


def fp16(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def weights_abi(dim):
    return to_abi(dim, oracle.lattice(dim)[1])


def refs16(params, phi, p):
    """(P, F, s): the references a cell writes with (fp16 of its p* and phi)
    and its flow scale rho(F) cs^2."""
    P, F = fp16(p), fp16(phi)
    s = (params["rho_l"] + (params["rho_h"] - params["rho_l"]) * F) / 3.0
    return P, F, s


def flow_q(dim, pops_abi, refs, src):
    """Codes of the moving flow directions (library order; rest row zero) and
    the per-element change one FP16 step of the writer's references makes."""
    P, F, s = refs
    w = weights_abi(dim)
    Q = pops_abi.shape[0]
    q = np.zeros_like(pops_abi)
    dref = np.zeros_like(pops_abi)
    for a in range(Q):
        if a == Q // 2:
            continue
        Pa, Fa, sa = (P.ravel()[src[a]], F.ravel()[src[a]], s.ravel()[src[a]])
        q[a] = (pops_abi[a] / w[a] - Pa) / sa
        dref[a] = ulp16(Pa) / sa + np.abs(q[a]) * ulp16(Fa) / (3 * sa)
    return q, dref


def phase_q(dim, pops_abi, F):
    """Codes of the moving phase-field directions (reader-referenced)."""
    w = weights_abi(dim)
    Q = pops_abi.shape[0]
    q = np.zeros_like(pops_abi)
    for a in range(Q):
        if a != Q // 2:
            q[a] = pops_abi[a] / w[a] - F
    return q, np.broadcast_to(ulp16(F), q.shape) * (np.arange(Q) != Q // 2).reshape(
        (-1,) + (1,) * (q.ndim - 1))


def check_q(q_gpu, q_or, slack):
    """Within one FP16 ulp of the code plus slack (array or scalar)."""
    bound = np.maximum(ulp16(q_or), ulp16(q_gpu)) + slack
    excess = np.abs(q_gpu - q_or) - bound
    assert excess.max() <= 0, (np.abs(q_gpu - q_or).max(), float(excess.max()))
    # most values round to the same FP16 number
    assert np.mean(np.abs(q_gpu - q_or) <= 0.5 * ulp16(q_or) + slack) > 0.99


def by_writer(dim, d_abi, src):
    """Per cell x: the sum over the moving directions of d at the cells that
    pull what x wrote (library order)."""
    Q = d_abi.shape[0]
    out = np.zeros(d_abi[0].size)
    for a in range(Q):
        if a != Q // 2:
            np.add.at(out, src[a].ravel(), d_abi[a].ravel())
    return out.reshape(d_abi.shape[1:])


def check_rest_remainder(dim, got, want, src):
    """The FP32 rest direction holds the remainder of the writer's zeroth
    moment over the values its readers decode, so the rounding of the moving
    values a cell wrote reappears, with the other sign, in its rest value:
    rest error + sum of its moving values' errors = the zeroth moment's own
    FP32 error."""
    Q = got.shape[0]
    d = got - want
    total = d[Q // 2] + by_writer(dim, d, src)
    assert np.abs(total).max() < 1e-5 * np.abs(want).max(), np.abs(total).max()


def check_fp16_step(dim, params, got_f, got_g, f1, g1, fl, storage):
    """One-step comparison in the stored representation; fl: the oracle's
    fields of the level the step started from (the writers' references)."""
    Q = got_f.shape[0]
    src = source_cells(dim, params["n"], params["bc"])
    refs = refs16(params, fl["phi"], fl["p"])
    fo = to_abi(dim, f1)
    qo, dref = flow_q(dim, fo, refs, src)
    qg, _ = flow_q(dim, got_f, refs, src)
    w = weights_abi(dim).reshape((-1,) + (1,) * (fo.ndim - 1))
    s_src = refs[2].ravel()[src]
    fp32 = 4e-6 * np.abs(fo).max() / (w * s_src)
    check_q(qg, qo, fp32 + dref)
    check_rest_remainder(dim, got_f, fo, src)
    go = to_abi(dim, g1)
    if storage == "fp16s":
        assert rel_err(got_g, go) < 2e-6
    else:
        qo, dref = phase_q(dim, go, refs[1])
        qg, _ = phase_q(dim, got_g, refs[1])
        check_q(qg, qo, 4e-6 * (np.abs(qo).max() + 1.0) + dref)
        check_rest_remainder(dim, got_g, go, src)


@pytest.mark.parametrize("storage", ["fp16s", "fp16s_all"])
@pytest.mark.parametrize("dim,n,bc", CONFIGS)
def test_one_step_in_stored_representation(storage, dim, n, bc):
    params, phi, u, p = random_case(dim, n, bc, seed=5)
    po, f, g = noisy_state(params, phi, u, p, seed=9, amp=0.03)
    s = mplb.Solver(params, storage=storage)
    s.init(phi, u, p)
    s.set_populations(0, to_abi(dim, f))
    s.set_populations(1, to_abi(dim, g))
    f0 = from_abi(dim, s.get_populations(0))  # the state the GPU holds, decoded
    g0 = from_abi(dim, s.get_populations(1))
    s.step(1)
    f1, g1 = oracle.step(po, f0, g0, 1)
    fl = oracle.fields(po, f0, g0)  # time level n: the references the writers use
    check_fp16_step(dim, params, s.get_populations(0), s.get_populations(1), f1, g1, fl, storage)


@pytest.mark.parametrize("storage", ["fp16s", "fp16s_all"])
def test_init_encodes_the_equilibrium_to_fp16(storage):
    case = inputs.rti3d(nx=16, ny=12, nz=24, amp=1.5)
    po = oracle.params_from_dict(case.params)
    f, g = oracle.init(po, case.phi, case.u, case.p)
    s = mplb.Solver(case.params, storage=storage)
    s.init(case.phi, case.u, case.p)
    # the initial state's references: the prescribed fields
    src = source_cells(3, case.params["n"], case.params["bc"])
    refs = refs16(case.params, case.phi, case.p)
    qo, dref = flow_q(3, to_abi(3, f), refs, src)
    qg, _ = flow_q(3, s.get_populations(0), refs, src)
    check_q(qg, qo, 4e-6 * np.abs(qo).max() + dref)
    if storage == "fp16s_all":
        qo, dref = phase_q(3, to_abi(3, g), refs[1])
        qg, _ = phase_q(3, s.get_populations(1), refs[1])
        check_q(qg, qo, 4e-6 * (np.abs(qo).max() + 1.0) + dref)


def fp16_floor(po, f, g, steps, seed=0):
    """Oracle-vs-oracle field differences after `steps` when, after every
    step, each flow population's deviation from w p (and, for the phase-field
    set, from w phi) carries a relative perturbation of one FP16 ulp."""
    rng = np.random.default_rng(seed)
    fa, ga = oracle.step(po, f, g, steps)
    w = oracle.lattice(po.dim)[1]
    shape = (-1,) + (1,) * (f.ndim - 1)
    wb = np.asarray(w).reshape(shape)
    fb, gb = f, g
    for _ in range(steps):
        fb, gb = oracle.step(po, fb, gb, 1)
        fl = oracle.fields(po, fb, gb)
        df = fb - wb * fl["p"]
        dg = gb - wb * fl["phi"]
        fb = wb * fl["p"] + df * (1 + 2.0 ** -11 * rng.uniform(-1, 1, fb.shape))
        gb = wb * fl["phi"] + dg * (1 + 2.0 ** -11 * rng.uniform(-1, 1, gb.shape))
    A, B = oracle.fields(po, fa, ga), oracle.fields(po, fb, gb)
    return A, {k: np.abs(A[k] - B[k]).max() for k in ("phi", "u", "p")}


@pytest.mark.parametrize("storage", ["fp16s", "fp16s_all"])
def test_c1_rayleigh_taylor_fp16_within_fp16_floor(storage):
    # 2-D Rayleigh-Taylor, 64 x 256, At 0.5, Re 256, 2000 steps
    case = inputs.rti2d()
    po = oracle.params_from_dict(case.params)
    f, g = oracle.init(po, case.phi, case.u, case.p)
    ref, floor = fp16_floor(po, f, g, case.steps)
    s = mplb.Solver(case.params, storage=storage)
    s.init(case.phi, case.u, case.p)
    s.step(case.steps)
    got = s.fields()
    diff = {k: np.abs(got[k] - ref[k]).max() for k in ("phi", "u", "p")}
    print("C1 %s 2000 steps: gpu-oracle %s, FP16 floor %s" % (storage, diff, floor))
    for k in diff:
        assert diff[k] < 5 * floor[k], (k, diff[k], floor[k])
    red, rc = s.reduce()
    assert rc == mplb.OK
    m0 = case.phi.sum()
    drift = abs(red[0] - m0) / m0
    print("C1 %s phase-mass drift %.3e" % (storage, drift))
    # the rest direction (FP32) is the remainder of the phase mass over the
    # values the readers decode: exact to FP32 round-off in both formats
    assert drift < 1e-6
