"""The allocation-free reduction (mplb_reduce_noalloc) against mplb_reduce:
the same kernels over the library's static device scratch instead of the
solver's arena, so the same bits; two calls in a row, the second on a
smaller lattice (the scratch keeps the first call's contents)."""
import numpy as np
import pytest

from paper_2101_06769_amd import inputs
from tests.helpers import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2101_06769_amd import mplb


def _solver(nx, ny, nz, storage):
    case = inputs.rti3d(nx=nx, ny=ny, nz=nz, amp=1.5)
    s = mplb.Solver(case.params, storage=storage)
    s.init(case.phi, case.u, case.p)
    s.step(5)
    return s


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16s_all"])
def test_noalloc_reduce_equals_reduce_twice_second_smaller(storage):
    big = _solver(128, 64, 96, storage)      # 786432 cells: every one of the 1024 blocks
    small = _solver(16, 8, 24, storage)      # 3072 cells: 12 blocks
    for s in (big, small):
        want, rc_want = s.reduce()
        got, rc_got = s.reduce_noalloc()
        assert rc_got == rc_want == mplb.OK
        assert np.array_equal(got, want), (got, want)
    # and a non-finite state is reported the same way
    case = inputs.rti3d(nx=16, ny=8, nz=24, amp=1.5)
    phi = case.phi.copy()
    phi[3, 2, 1] = np.nan
    s = mplb.Solver(case.params, storage=storage)
    s.init(phi, case.u, case.p)
    _, rc = s.reduce_noalloc()
    assert rc == mplb.EUNSTABLE
