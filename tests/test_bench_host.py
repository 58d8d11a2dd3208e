"""Host logic of bench.py (CPU): the tensor spectrum mirrored from its stored
octant, used by the informational rocFFT and host-FFT lines, equals the full
half-spectrum of a real tensor with the demagnetization tensor's parities
(xx, yy, zz even in every axis; xy odd in x and y; xz in x and z; yz in y and
z), whose transform is real."""
import numpy as np
import pytest

import bench


@pytest.mark.parametrize("P", [(8, 6, 10), (16, 12, 6), (4, 2, 2)])
def test_mirrored_spectrum_equals_full_half_spectrum(P):
    Px, Py, Pz = P
    rng = np.random.default_rng(sum(P))
    odd = [(0, 0, 0), (0, 0, 0), (0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    N = np.zeros((6, Pz, Py, Px))
    for c, (ox, oy, oz) in enumerate(odd):
        a = rng.standard_normal((Pz, Py, Px))
        for ax, o in ((2, ox), (1, oy), (0, oz)):  # f(-u) = (-1)^o f(u) on the periodic grid
            a = 0.5 * (a + (-1) ** o * np.roll(np.flip(a, axis=ax), 1, axis=ax))
        N[c] = a
    F = np.fft.rfftn(N, axes=(1, 2, 3))
    assert np.abs(F.imag).max() < 1e-12
    octant = np.ascontiguousarray(F.real[:, :Pz // 2 + 1, :Py // 2 + 1, :].transpose(2, 0, 3, 1))
    full = bench.mirrored_spectrum(np, octant, Py, Pz)
    assert full.shape == (6, Pz, Py, Px // 2 + 1)
    assert np.abs(full - F.real).max() < 1e-12


def test_union_of_kernel_intervals():
    """The busy time of a profiled range: overlapping dispatches (concurrent
    streams) count once, gaps not at all."""
    assert bench._union_ns([]) == 0
    assert bench._union_ns([(0, 10)]) == 10
    assert bench._union_ns([(5, 15), (0, 10), (20, 30)]) == 25
    assert bench._union_ns([(0, 100), (10, 20), (30, 40)]) == 100
    assert bench._union_ns([(0, 10), (10, 20)]) == 20
