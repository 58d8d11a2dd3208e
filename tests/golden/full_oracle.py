"""Whole-grid oracle fields of two workloads, kept in a cache of this folder.

The direct O(N^2) sums over every cell take minutes of host time at these
sizes, so the GPU tests read them from here.  This script calls only the
oracle (``oracle/``) and the seeded input generators; nothing in a cached
file comes from the HIP path.  Each file carries the key it was written for
(workload parameters and the oracle source's hash) and is recomputed when
the key differs or the file is missing.

Workloads:
  random_128x128x32   128 x 128 x 32 cubic cells of 2.5 nm, Ms = 8e5 A/m,
                      i.i.d. random unit m (seed 2), FP32-representable:
                      the forward field H = -Ms N * m (Sec. 3.1, eq. (demag)).
  strip_512x128x4     512 x 128 x 4 cells of 1.95 x 1.95 x 0.75 nm,
                      Ms = 8e5 A/m, m = normalise((1, 0.1, 0) + 0.2 xi)
                      (seed 5) and a cotangent g (standard normal, seed 51),
                      both FP32-representable: the forward field and the
                      transposed operator applied to g, each as its own sum.

  python tests/golden/full_oracle.py      (writes both; about 8 minutes on 8 threads)
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CACHE = os.path.join(HERE, "full")

WORKLOADS = {
    "random_128x128x32": {"shape": (128, 128, 32), "cell": (2.5e-9, 2.5e-9, 2.5e-9), "Ms": 8e5,
                          "m": ("random_unit", 2), "g": None},
    "strip_512x128x4": {"shape": (512, 128, 4), "cell": (1.95e-9, 1.95e-9, 0.75e-9), "Ms": 8e5,
                        "m": ("noisy_strip", 5), "g": ("normal", 51)},
}


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


def inputs_of(name):
    """(m, g) of a workload, FP32-representable float64 arrays (g may be None)."""
    from paper_1204_4302_amd import inputs
    w = WORKLOADS[name]
    shape = w["shape"]
    kind, seed = w["m"]
    m = _f32(getattr(inputs, kind)(shape, seed))
    g = None
    if w["g"] is not None:
        nx, ny, nz = shape
        g = _f32(np.random.default_rng(w["g"][1]).standard_normal((3, nz, ny, nx)))
    return m, g


def _key(name):
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "oracle", "demag_oracle.c"), "rb") as f:
        h.update(f.read())
    w = WORKLOADS[name]
    return f"{name} {w['shape']} {w['cell']} {w['Ms']} {w['m']} {w['g']} oracle={h.hexdigest()[:16]}"


def _path(name):
    return os.path.join(CACHE, name + ".npz")


def load(name, compute=True):
    """dict(m, g, H, HT) of a workload from the cache, computing (and caching)
    it when missing or stale; None if not cached and compute is False."""
    path = _path(name)
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            if str(z["key"]) == _key(name):
                return {k: z[k] for k in ("m", "g", "H", "HT") if k in z.files}
    if not compute:
        return None
    return write(name)


def write(name):
    import oracle
    w = WORKLOADS[name]
    m, g = inputs_of(name)
    o = oracle.Oracle(w["shape"], w["cell"])
    out = {"m": m, "H": o.field(m, w["Ms"])}
    if g is not None:
        out["g"] = g
        out["HT"] = o.field_T(g, w["Ms"])
    os.makedirs(CACHE, exist_ok=True)
    tmp = _path(name) + ".tmp.npz"
    np.savez(tmp, key=np.array(_key(name)), **out)
    os.replace(tmp, _path(name))
    return out


if __name__ == "__main__":
    import time
    for name in (sys.argv[1:] or list(WORKLOADS)):
        t0 = time.perf_counter()
        write(name)
        print(f"{name}: {time.perf_counter() - t0:.1f} s", flush=True)
