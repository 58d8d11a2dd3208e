"""GPU parity: the HIP path against the CPU oracle, element by element.

Bars (relative max-norm, eps = max|H - H_ref| / max|H_ref|): FP64 <= 1e-12,
FP32 <= 1e-5.  Shapes span several workgroup tiles and ragged tails, padded
lengths with radix-3/5 factors, degenerate axes of length 1 and non-cubic
cells.  FP32 inputs are compared against the oracle evaluated on the same
FP32-rounded m promoted to FP64, so input quantisation is not counted.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_4302_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def rel_err(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def to_gpu(m, dtype):
    return torch.from_numpy(np.ascontiguousarray(m)).to(device="cuda", dtype=dtype)


def quantised(m, dtype):
    return m.astype(np.float32).astype(np.float64) if dtype == torch.float32 else m


_ORACLES = {}


def get_oracle(shape, cell):
    key = (tuple(shape), tuple(cell))
    if key not in _ORACLES:
        _ORACLES[key] = oracle.Oracle(shape, cell)
    return _ORACLES[key]


_PLANS = {}


def get_plan(shape, cell, dtype):
    from paper_1204_4302_amd import Plan
    key = (tuple(shape), tuple(cell), dtype)
    if key not in _PLANS:
        _PLANS[key] = Plan(shape, cell, dtype)
    return _PLANS[key]


SHAPES = [
    ((8, 8, 8), (2e-9, 2e-9, 2e-9), 8e5),          # the plain FP64 DM case
    ((1, 1, 1), (2e-9, 2e-9, 3e-9), 1.4e6),        # single cell
    ((5, 1, 1), (2e-9, 2e-9, 2e-9), 8e5),          # chain
    ((1, 1, 7), (1.95e-9, 1.95e-9, 0.75e-9), 8e5),  # column
    ((13, 7, 5), (2e-9, 2e-9, 3e-9), 1.4e6),       # non-smooth n -> padded 30, 14, 10
    ((24, 17, 3), (1.95e-9, 1.95e-9, 0.75e-9), 8e5),
    ((33, 20, 9), (2.5e-9, 2.5e-9, 2.5e-9), 8e5),  # padded 72 (8*9) ragged tiles
    ((48, 12, 6), (2e-9, 2e-9, 2e-9), 8e5),        # 96 = 8*4*3
    ((70, 9, 2), (2e-9, 3e-9, 1e-9), 8e5),         # far band reached along x
    ((64, 32, 8), (2e-9, 2e-9, 3e-9), 1.4e6),      # power-of-two padded lengths 128, 64, 16
    ((16, 128, 32), (2.5e-9, 2.5e-9, 2.5e-9), 8e5),  # 32, 256, 64
    ((4, 4, 64), (1.95e-9, 1.95e-9, 0.75e-9), 8e5),  # 8, 8, 128: thin pencils in x and y
    ((2, 3, 4), (2e-9, 2e-9, 2e-9), 8e5),          # 4, 6 (generic), 8
    ((29, 61, 11), (2e-9, 2e-9, 3e-9), 1.4e6),     # 64 (p2, 29 valid), 128 (p2, 61 valid), 24: ragged tiles
    ((47, 11, 23), (2e-9, 2e-9, 3e-9), 1.4e6),     # 96, 24, 48 = 3 * 2^a, all ragged (47, 11, 23 valid)
]


@pytest.mark.parametrize("shape,cell,Ms", SHAPES, ids=lambda v: str(v))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_field_random_vs_oracle(shape, cell, Ms, dtype):
    o = get_oracle(shape, cell)
    plan = get_plan(shape, cell, dtype)
    m = inputs.random_unit(shape, 1)
    H = plan.field(to_gpu(m, dtype), Ms).double().cpu().numpy()
    ref = o.field(quantised(m, dtype), Ms)
    err = rel_err(H, ref)
    print(f"shape={shape} dtype={dtype} rel_err={err:.3e}")
    assert err <= (FP64_TOL if dtype == torch.float64 else FP32_TOL)


@pytest.mark.parametrize("shape,cell,Ms", [((64, 32, 8), (2e-9, 2e-9, 3e-9), 1.4e6),
                                            ((29, 61, 11), (2e-9, 2e-9, 3e-9), 1.4e6),
                                            ((47, 11, 23), (2e-9, 2e-9, 3e-9), 1.4e6)], ids=str)
def test_generic_and_pow2_kernels_agree(shape, cell, Ms):
    """Both kernel families on one plan: each within the bar of the oracle."""
    from paper_1204_4302_amd import Plan
    o = get_oracle(shape, cell)
    m = inputs.random_unit(shape, 4)
    ref = o.field(m, Ms)
    for generic in (1, 0):
        plan = Plan(shape, cell, torch.float64)
        plan.set_option("generic_kernels", generic)
        H = plan.field(to_gpu(m, torch.float64), Ms).cpu().numpy()
        assert rel_err(H, ref) <= FP64_TOL
        plan.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_uniform_cube_state(dtype):
    shape, cell, Ms = (8, 8, 8), (2e-9,) * 3, 8e5
    o = get_oracle(shape, cell)
    plan = get_plan(shape, cell, dtype)
    m = inputs.uniform(shape, (1, 1, 1))
    H = plan.field(to_gpu(m, dtype), Ms).double().cpu().numpy()
    ref = o.field(quantised(m, dtype), Ms)
    assert rel_err(H, ref) <= (FP64_TOL if dtype == torch.float64 else FP32_TOL)


@pytest.mark.parametrize("shape,cell", [((8, 8, 8), (2e-9,) * 3), ((70, 9, 2), (2e-9, 3e-9, 1e-9)),
                                        ((60, 60, 4), (1.95e-9, 1.95e-9, 0.75e-9)),
                                        ((64, 10, 6), (2e-9, 2e-9, 3e-9))])
def test_tensor_octant_per_band(shape, cell):
    """FP64 setup tensor vs the binary128 f/g oracle, offset by offset."""
    o = get_oracle(shape, cell)
    plan = get_plan(shape, cell, torch.float64)
    N = plan.tensor()
    ref = o.Noct
    scale = np.max(np.abs(ref), axis=0)  # per offset
    err = np.max(np.abs(N - ref), axis=0) / scale
    nx, ny, nz = shape
    h = max(cell)
    oz, oy, ox = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rho = np.sqrt((ox * cell[0]) ** 2 + (oy * cell[1]) ** 2 + (oz * cell[2]) ** 2) / h
    cheb = np.maximum(np.maximum(ox, oy), oz)
    for name, mask in [("near", cheb <= 1), ("mid", (cheb > 1) & (rho < 40)), ("far", rho >= 40)]:
        if mask.any():
            print(f"{shape} {name}: max rel err {err[mask].max():.2e} over {mask.sum()} offsets")
            assert err[mask].max() <= 1e-12


def test_spectrum_matches_fft_of_oracle_tensor():
    """The stored FP64 spectrum equals -1/(PxPyPz) x DFT of the P-periodic
    embedding of the oracle tensor (numpy FFT), on the stored octant."""
    shape, cell = (12, 10, 6), (2e-9, 2e-9, 3e-9)
    o = get_oracle(shape, cell)
    plan = get_plan(shape, cell, torch.float64)
    info = plan.info()
    Px, Py, Pz, Kx = info["Px"], info["Py"], info["Pz"], info["Kx"]
    nx, ny, nz = shape
    par = [(0, 0, 0), (0, 0, 0), (0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    S = plan.spectrum()
    for c in range(6):
        A = np.zeros((Pz, Py, Px))
        for sz in (1, -1):
            for sy in (1, -1):
                for sx in (1, -1):
                    sign = (sx if par[c][0] else 1) * (sy if par[c][1] else 1) * (sz if par[c][2] else 1)
                    zi = (sz * np.arange(nz)) % Pz
                    yi = (sy * np.arange(ny)) % Py
                    xi = (sx * np.arange(nx)) % Px
                    A[np.ix_(zi, yi, xi)] = sign * o.Noct[c]
        F = np.fft.fftn(A)  # axes (z, y, x)
        ref = (-F.real / (Px * Py * Pz))[: Pz // 2 + 1, : Py // 2 + 1, :Kx]  # [kz][ky][kx]
        got = S[:, c, :, :].transpose(2, 0, 1)  # [ky][kx][kz] -> [kz][ky][kx]
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def _embedded(o, c, P):
    """Component c of the oracle tensor octant mirrored into a P-periodic
    array [Pz][Py][Px] with its parity signs (xy odd in x and y, xz in x and z,
    yz in y and z), zero in the padding gap."""
    Px, Py, Pz = P
    nz, ny, nx = o.Noct.shape[1:]
    par = [(0, 0, 0), (0, 0, 0), (0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    A = np.zeros((Pz, Py, Px))
    for sz in (1, -1):
        for sy in (1, -1):
            for sx in (1, -1):
                sign = (sx if par[c][0] else 1) * (sy if par[c][1] else 1) * (sz if par[c][2] else 1)
                A[np.ix_((sz * np.arange(nz)) % Pz, (sy * np.arange(ny)) % Py, (sx * np.arange(nx)) % Px)] = \
                    sign * o.Noct[c]
    return A


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_spectrum_equals_direct_dft(dtype):
    """The FFT engine (radix-2/3/5 generic passes along x and y, register
    kernel along z) against the DFT by its definition, sum_o A(o)
    exp(-2 pi i k.o / P) as explicit products with the DFT matrices, on the
    stored octant: the tensor spectrum of a 5-smooth grid (padded 30 x 18 x 8)."""
    shape, cell = (15, 9, 4), (2e-9, 2e-9, 3e-9)
    o = get_oracle(shape, cell)
    plan = get_plan(shape, cell, dtype)
    info = plan.info()
    P = (info["Px"], info["Py"], info["Pz"])
    assert P == (30, 18, 8)
    Kx, S = info["Kx"], plan.spectrum()

    def dft_matrix(n, keep):
        k = np.arange(keep)[:, None]
        t = np.arange(n)[None, :]
        return np.exp(-2j * np.pi * ((k * t) % n) / n)  # exact angle reduction before exp

    Wx, Wy, Wz = dft_matrix(P[0], Kx), dft_matrix(P[1], P[1] // 2 + 1), dft_matrix(P[2], P[2] // 2 + 1)
    for c in range(6):
        A = _embedded(o, c, P)
        F = np.einsum("az,by,cx,zyx->abc", Wz, Wy, Wx, A)  # [kz][ky][kx]
        ref = -F.real / (P[0] * P[1] * P[2])
        got = S[:, c, :, :].transpose(2, 0, 1)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"{dtype} component {c}: {err:.2e}")
        assert err <= (1e-13 if dtype == torch.float64 else 3e-7)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape,generic", [((13, 7, 5), False), ((24, 17, 3), True)], ids=["x30", "generic_kernels"])
def test_energy_vs_oracle_generic_x(dtype, shape, generic):
    """The energy epilogue of the generic X-C2R kernel: a 5-smooth padded x
    length (30), and a plan with generic_kernels = 1 on every pass."""
    cell, Ms = (2e-9, 2e-9, 3e-9), 8e5
    from paper_1204_4302_amd import Plan
    o = get_oracle(shape, cell)
    plan = Plan(shape, cell, dtype)
    if generic:
        plan.set_option("generic_kernels", 1)
    assert "generic" in plan.describe().split()[-1] or not generic
    for m in [inputs.random_unit(shape, 12), inputs.gaussian_vortex(shape, cell, 8e-9)]:
        mq = quantised(m, dtype)
        Href = o.field(mq, Ms)
        ref = o.energy(mq, Href, Ms)
        H, E = plan.field_energy(to_gpu(m, dtype), Ms)
        scale = 0.5 * oracle.MU0 * Ms * o.volume * np.sum(np.abs(mq * Href))
        tol = 1e-12 if dtype == torch.float64 else 1e-5
        print(f"{shape} generic={generic} {dtype}: |dE|/scale {abs(float(E) - ref) / scale:.2e}")
        assert abs(float(E) - ref) <= tol * scale
        assert rel_err(H.double().cpu().numpy(), Href) <= (FP64_TOL if dtype == torch.float64 else FP32_TOL)
    plan.close()


def test_plan_busy_on_another_stream_is_estate():
    """A plan runs on one stream at a time: a call on stream B while the
    plan's work on stream A is still pending returns DEMAG_ESTATE (the work on
    A is held back by a bounded spin kernel queued before it); once A has
    drained, stream B may use the plan."""
    from paper_1204_4302_amd import Plan
    from paper_1204_4302_amd._lib import DemagError
    shape, cell = (64, 32, 16), (2e-9, 2e-9, 3e-9)
    plan = Plan(shape, cell, torch.float32)
    m = to_gpu(inputs.random_unit(shape, 13), torch.float32)
    H0 = plan.field(m, 8e5)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(sa):
        torch.cuda._sleep(100_000_000)  # bounded spin: a few tens of ms
        plan.field(m, 8e5)
    with torch.cuda.stream(sb):
        with pytest.raises(DemagError, match="ESTATE"):
            plan.field(m, 8e5)
    sa.synchronize()
    with torch.cuda.stream(sb):
        H = plan.field(m, 8e5)
    sb.synchronize()
    assert torch.equal(H, H0)
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_energy_vs_oracle(dtype):
    shape, cell, Ms = (24, 17, 3), (1.95e-9, 1.95e-9, 0.75e-9), 8e5
    o = get_oracle(shape, cell)
    plan = get_plan(shape, cell, dtype)
    for m in [inputs.uniform(shape, (1, 0.2, 0.1)), inputs.gaussian_vortex(shape, cell, 10e-9),
              inputs.random_unit(shape, 5)]:
        mq = quantised(m, dtype)
        ref = o.energy(mq, o.field(mq, Ms), Ms)
        H, E = plan.field_energy(to_gpu(m, dtype), Ms)
        E = float(E.cpu())
        # scale for states whose energy nearly cancels: (mu0/2) Ms V sum |m||H|
        Href = o.field(mq, Ms)
        scale = 0.5 * oracle.MU0 * Ms * o.volume * np.sum(np.abs(mq * Href))
        tol = 1e-12 if dtype == torch.float64 else 1e-5
        assert abs(E - ref) <= tol * scale
        assert abs(plan.energy(to_gpu(m, dtype), Ms) - ref) <= tol * scale  # the energy alone
        assert rel_err(H.double().cpu().numpy(), Href) <= (FP64_TOL if dtype == torch.float64 else FP32_TOL)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_adjoint_vs_oracle_transpose(dtype):
    shape, cell, Ms = (16, 8, 2), (1.95e-9, 1.95e-9, 0.75e-9), 8e5
    o = get_oracle(shape, cell)
    plan = get_plan(shape, cell, dtype)
    g = np.random.default_rng(6).standard_normal((3, 2, 8, 16))
    ref = o.field_T(quantised(g, dtype), Ms)
    got = plan.adjoint(to_gpu(g, dtype), Ms).double().cpu().numpy()
    assert rel_err(got, ref) <= (FP64_TOL if dtype == torch.float64 else FP32_TOL)
    # accumulate flag: gm += A^T gH
    base = np.random.default_rng(7).standard_normal(g.shape)
    acc = to_gpu(base, dtype)
    plan.adjoint(to_gpu(g, dtype), Ms, out=acc, accumulate=True)
    assert rel_err(acc.double().cpu().numpy(), quantised(base, dtype) + ref) <= (
        FP64_TOL if dtype == torch.float64 else FP32_TOL)


def test_repeatable_bitwise():
    shape, cell, Ms = (33, 20, 9), (2.5e-9,) * 3, 8e5
    plan = get_plan(shape, cell, torch.float32)
    m = to_gpu(inputs.random_unit(shape, 9), torch.float32)
    a = plan.field(m, Ms).cpu()
    b = plan.field(m, Ms).cpu()
    assert torch.equal(a, b)
    _, e1 = plan.field_energy(m, Ms)
    _, e2 = plan.field_energy(m, Ms)
    assert float(e1) == float(e2)


def test_sentinels_around_output():
    """Writes stay inside H: guard bands before and after it are untouched."""
    shape, cell, Ms = (13, 7, 5), (2e-9, 2e-9, 3e-9), 1.4e6
    plan = get_plan(shape, cell, torch.float32)
    n = 3 * 13 * 7 * 5
    buf = torch.full((n + 2048,), 12345.0, device="cuda", dtype=torch.float32)
    H = buf[1024:1024 + n].view(3, 5, 7, 13)
    plan.field(to_gpu(inputs.random_unit(shape, 2), torch.float32), Ms, out=H)
    torch.cuda.synchronize()
    assert torch.all(buf[:1024] == 12345.0) and torch.all(buf[1024 + n:] == 12345.0)


@pytest.mark.parametrize("shape,cell", [((16, 16, 8), (10e-9, 10e-9, 1e-9)), ((24, 6, 4), (1e-9, 1e-9, 10e-9)),
                                        ((48, 48, 4), (5e-9, 5e-9, 0.5e-9))], ids=lambda v: str(v))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_flat_and_elongated_cells_vs_oracle(shape, cell, dtype):
    """Cells with a 10:1 and a 1:10 aspect ratio: the tensor's distance bands
    (reduced units of the largest edge; far-field series beyond 40 of them,
    Gauss-Legendre in between) against the binary128 oracle tensor."""
    o = get_oracle(shape, cell)
    plan = get_plan(shape, cell, dtype)
    m = inputs.random_unit(shape, 5)
    ref = o.field(quantised(m, dtype), 8e5)
    H = plan.field(to_gpu(m, dtype), 8e5).double().cpu().numpy()
    err = float(np.abs(H - ref).max() / np.abs(ref).max())
    print(f"{shape} {cell} {dtype}: {err:.2e}")
    assert err <= (1e-12 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_cell_scale_invariance(dtype):
    """The tensor depends on the cell's shape only (lengths reduced by the
    largest edge): cells scaled by 2^10 (exact in binary, so the reduced edges
    are the same numbers) give the same field bit for bit, and an energy
    larger by exactly the volume ratio 2^30."""
    from paper_1204_4302_amd import Plan
    shape = (24, 17, 3)
    small = (1.95e-9, 1.95e-9, 0.75e-9)
    big = tuple(c * 1024 for c in small)
    m = to_gpu(inputs.random_unit(shape, 9), dtype)
    H1, E1 = Plan(shape, small, dtype).field_energy(m, 8e5)
    H2, E2 = Plan(shape, big, dtype).field_energy(m, 8e5)
    assert torch.equal(H1, H2)
    print(f"{dtype}: energy ratio {float(E2) / float(E1)!r}")
    assert float(E2) == float(E1) * 2.0 ** 30


# padded z: 6 (3 * 2^a; FP64 on the generic Z pass), 128, 24, 4096 (split
# form), 10 (generic), 2 (one cell along z); one cell, and one cell along x
# (padded x 2: every kx is 0 or the Nyquist frequency)
ENERGY_ONLY = [((24, 17, 3), (1.95e-9, 1.95e-9, 0.75e-9)), ((16, 8, 64), (2e-9, 2e-9, 3e-9)),
               ((9, 6, 12), (2e-9, 2e-9, 2e-9)), ((2, 2, 2048), (2e-9, 2e-9, 1e-9)),
               ((13, 7, 5), (2e-9, 3e-9, 2e-9)), ((7, 5, 1), (2e-9, 2e-9, 2e-9)),
               ((1, 1, 1), (2e-9, 2e-9, 2e-9)), ((1, 6, 4), (2e-9, 2e-9, 2e-9))]


@pytest.mark.parametrize("shape,cell", ENERGY_ONLY, ids=lambda v: str(v))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_energy_alone_vs_oracle(shape, cell, dtype):
    """demag_energy without a field: with the register Z pass, three passes and
    the spectral sum of Re(M^H Nhat M) (Parseval on the padded grid); with the
    generic Z pass, the five passes and the sum of m.H.  Both against the
    oracle's energy at 1e-12 / 1e-5 of (mu0/2) Ms V sum |m.H|; the path taken
    is seen in pass timing, which records field evaluations only."""
    from paper_1204_4302_amd import Plan
    Ms = 8e5
    o = get_oracle(shape, cell)
    plan = Plan(shape, cell, dtype)
    info = plan.info()
    z_register = "z_conv:pow2" in plan.describe()  # the register kernels (powers of two and 3 * 2^a)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for seed in (21, 22):
        m = inputs.random_unit(shape, seed)
        mq = quantised(m, dtype)
        Href = o.field(mq, Ms)
        ref = o.energy(mq, Href, Ms)
        scale = 0.5 * oracle.MU0 * Ms * o.volume * np.sum(np.abs(mq * Href))
        plan.set_option("pass_timing", 4)
        E = plan.energy(to_gpu(m, dtype), Ms)
        _, recorded = plan.pass_times()
        plan.set_option("pass_timing", 0)
        print(f"{shape} {dtype} padded z {info['Pz']}: {plan.describe().split(' ')[2]}; "
              f"E {E:.9e} oracle {ref:.9e}, err/scale {abs(E - ref) / scale:.2e}, recorded {recorded}")
        assert abs(E - ref) <= tol * scale
        assert recorded == (0 if z_register else 1)
    plan.close()
