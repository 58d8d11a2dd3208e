"""MI355X-native demagnetization-tensor (DM) stray-field solver.

H = -Ms N * m on a regular cuboid grid (Abert et al., arXiv:1204.4302,
Sec. 3.1), evaluated by hand-written gfx950 HIP kernels behind a C ABI
(include/demag.h).  Import the GPU classes from here; the submodule `inputs`
(seeded synthetic states) needs neither torch nor the library.
"""
__all__ = ["Plan", "Batch", "DemagField", "DemagEnergy", "demag_field", "demag_energy", "MU0", "TUCKER", "CP"]


def __getattr__(name):
    if name in __all__:
        from . import plan as _plan
        return getattr(_plan, name)
    raise AttributeError(name)
