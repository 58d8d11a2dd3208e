"""Closed forms the tests check against (independent of the oracle and of the
GPU path): demagnetizing factors of a uniformly magnetized cuboid."""
import mpmath as mp


def aharoni_dz(a, b, c):
    """D_z of a uniformly magnetized 2a x 2b x 2c prism (c along z), from
    Aharoni, J. Appl. Phys. 83, 3432 (1998), evaluated in 40-digit arithmetic."""
    with mp.workdps(40):
        a, b, c = mp.mpf(a), mp.mpf(b), mp.mpf(c)
        r = mp.sqrt(a * a + b * b + c * c)
        ab, bc, ac = mp.sqrt(a * a + b * b), mp.sqrt(b * b + c * c), mp.sqrt(a * a + c * c)
        t = ((b * b - c * c) / (2 * b * c) * mp.log((r - a) / (r + a))
             + (a * a - c * c) / (2 * a * c) * mp.log((r - b) / (r + b))
             + b / (2 * c) * mp.log((ab + a) / (ab - a))
             + a / (2 * c) * mp.log((ab + b) / (ab - b))
             + c / (2 * a) * mp.log((bc - b) / (bc + b))
             + c / (2 * b) * mp.log((ac - a) / (ac + a))
             + 2 * mp.atan(a * b / (c * r))
             + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
             + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
             + c / (a * b) * (ac + bc)
             - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
        return float(t / mp.pi)


def body_factors(lx, ly, lz):
    """(Dx, Dy, Dz) of an lx x ly x lz box by axis permutation of aharoni_dz."""
    a, b, c = lx / 2, ly / 2, lz / 2
    return aharoni_dz(b, c, a), aharoni_dz(c, a, b), aharoni_dz(a, b, c)
