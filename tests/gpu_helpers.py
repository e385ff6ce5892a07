"""Shared helpers for the GPU parity tests (oracle side in float64, GPU side through the C ABI)."""
import sys

import numpy as np

from oracle import evolve as oev
from oracle import propagate as opr
from oracle import screens as osc

TOL = 1e-4  # field relative-L2 bound against the FP64 oracle (complex64 path)


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def oracle_screens(path, seed, realizations, t=0):
    """Oracle screens [len(realizations)][M][N][N] for selected realizations only."""
    m, n = len(path.cn2dz), path.n
    out = np.empty((len(realizations), m, n, n))
    cache = {}
    for i, r in enumerate(realizations):
        for s in range(m):
            key = (r // 2, s)
            if key not in cache:
                cache[key] = osc.split_pair(osc.complex_screen(path, seed, t, r // 2, s))
            out[i, s] = cache[key][r % 2]
    return out


def oracle_propagate(path, seed, u0, realizations=None, screens=None, t=0):
    """Oracle fields (and checkpoints) for selected realizations."""
    if realizations is None:
        realizations = list(range(path.realizations))
    if screens is None:
        screens = oracle_screens(path, seed, realizations, t)
    u0 = np.asarray(u0, dtype=np.complex128)
    if u0.ndim == 3:
        u0 = u0[realizations]
    return opr.propagate(u0, path, screens)


def spectra_screens(spectra, r):
    return oev.screens_from_spectra(np.asarray(spectra, dtype=np.complex128), r)
