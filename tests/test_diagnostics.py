"""Host diagnostics (interface positions, spreading radius) on fields whose
answers are known exactly."""
import numpy as np

from paper_2101_06769_amd import diagnostics, inputs


def test_crossing_of_a_tanh_profile_is_its_centre():
    # linear interpolation between the bracketing cells: exact at a cell, and
    # within 1e-2 cells for W = 4 (the profile's curvature over one cell)
    z = np.arange(200, dtype=np.float64)
    for h in (50.0, 73.25, 120.6):
        phi = inputs.interface_profile(h - z, 4.0)  # heavy below h
        c = diagnostics.crossings(phi)
        assert len(c) == 1 and abs(c[0] - h) < 1e-2


def test_rti_positions_on_a_cosine_interface():
    case = inputs.rti2d(nx=64, ny=256, amp=5.0)
    spike, bubble = diagnostics.rti_positions(case.phi, 2)
    # interface y = 128 + 5 cos(2 pi x / 64): trough 123 at x = 32, crest 133 at x = 0
    assert abs(spike - 123.0) < 5e-3 and abs(bubble - 133.0) < 5e-3
    c3 = inputs.rti3d(nx=32, ny=32, nz=128, amp=3.0)
    spike, bubble = diagnostics.rti_positions(c3.phi, 3)
    assert abs(spike - (64.0 - 6.0)) < 5e-3 and abs(bubble - (64.0 + 6.0)) < 5e-3


def test_spreading_radius_of_a_slab():
    ny, nx = 40, 200
    x = np.arange(nx, dtype=np.float64)
    phi = np.zeros((1, ny, nx))
    r = 37.3
    phi[0, :, :] = inputs.interface_profile(r - np.abs(x - 100.0), 4.0)[None, :]
    assert abs(diagnostics.spreading_radius(phi, 100.0, 10.5) - r) < 1e-2
