"""Host-side pins of the tensor-grid (TG) quadrature (Sec. 3.2, eq.
(transform)): the Sinc nodes and weights the library builds must reproduce
1/r^3 = (4/sqrt(pi)) int_0^inf tau^2 exp(-tau^2 r^2) dtau, i.e.
1/r^3 ~ 4 pi sum_l w_l exp(-tau_l^2 r^2), over the whole distance range the
plan asks for, to the accuracy each precision's step promises."""
import numpy as np
import pytest

from paper_1204_4302_amd._lib import DemagError, load


def test_sinc_nodes_reproduce_inverse_cube():
    from paper_1204_4302_amd.plan import tg_sinc_nodes
    for step, tol in [(0.25, 5e-7), (0.15, 2e-12)]:
        rmin, rmax = 0.5, 400.0
        tau, w = tg_sinc_nodes(rmin, rmax, step)
        r = np.logspace(np.log10(rmin), np.log10(rmax), 2000)
        approx = 4 * np.pi * (w[None, :] * np.exp(-(tau[None, :] ** 2) * (r[:, None] ** 2))).sum(1)
        err = np.abs(approx * r ** 3 - 1).max()
        print(f"step {step}: {tau.size} nodes, max rel err {err:.2e}")
        assert err < tol
        assert np.all(np.diff(np.log(tau)) == pytest.approx(step, rel=1e-12))


def test_sinc_nodes_bad_arguments():
    lib = load()
    assert lib.demag_tg_sinc_nodes(0.0, 1.0, 0.2, None, None, 0) < 0
    assert lib.demag_tg_sinc_nodes(2.0, 1.0, 0.2, None, None, 0) < 0
    assert lib.demag_tg_sinc_nodes(1.0, 2.0, 0.0, None, None, 0) < 0
    from paper_1204_4302_amd.plan import tg_sinc_nodes
    with pytest.raises(DemagError):
        tg_sinc_nodes(1.0, 0.5, 0.2)


def test_tg_abi_null_arguments():
    lib = load()
    assert lib.demag_tg_prepare(None, None) == -1
    assert lib.demag_tg_field(None, None, 1.0, None, None) == -1
    assert lib.demag_tg_field_energy(None, None, 1.0, None, None, None) == -1
    assert lib.demag_tg_info(None, None) == -1
