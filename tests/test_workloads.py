"""The input generator (CPU only): the device-side evaluation of the analytic
initial fields (each vortex, pulse and ring on its bounding box, used for
meshes of ~1e9 nodes) equals the plain evaluation everywhere, and the
configurations have the geometry they state."""
import numpy as np
import pytest

from paper_2004_14887_amd import workloads as W

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("make", [
    lambda: W.rings_4level(seed=5, n0=32, sides=(22, 30, 32), steps=2, n_rings=4, n_pulses=2),
    lambda: W.rings_4level(seed=7, n0=48, sides=(30, 40, 44), steps=2, n_rings=6, n_pulses=3),
    lambda: W.pulse_vortices_3level(seed=2, n0=128, steps=2),
    lambda: W.pulse_ring_3d(seed=3, n0=32),
    lambda: W.vortex_2level(n0=64)])
def test_device_fields_equal_plain_fields(make):
    wl = make()
    peak = max(np.abs(W.initial_fields(wl, l)[1]).max() for l in range(wl.n_levels))
    for l in range(wl.n_levels):
        r0, u0 = W.initial_fields(wl, l)
        r1, u1 = W.initial_fields_device(wl, l, "cpu", slab_nodes=4096)
        # outside its box a structure contributes less than e^-32 times a
        # polynomial factor of its peak: 1e-12 of the peak bounds the cut
        assert np.abs(r1.numpy() - r0).max() <= 1e-14
        assert np.abs(u1.numpy() - u0).max() <= 1e-12 * peak


def test_four_level_mesh_fractions():
    """The 4-level 512^3 mesh: refined boxes of 30.3%, 10.0% and 1.87% of the
    volume (344, 238 and 136 coarse cells per side)."""
    wl = W.rings_4level(seed=5, steps=1)
    side0 = [wl.boxes[0][1][0] - wl.boxes[0][0][0]]
    for k in (1, 2):
        side0.append((wl.boxes[k][1][0] - wl.boxes[k][0][0]) / 2 ** k)
    frac = [(s / 512.0) ** 3 for s in side0]
    assert side0 == [344, 238, 136]
    assert abs(frac[0] - 0.303) < 1e-3 and abs(frac[1] - 0.100) < 1e-3 and abs(frac[2] - 0.0187) < 1e-4
    assert wl.dims(3) == (1089, 1089, 1089)
