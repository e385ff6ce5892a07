"""Screen placement along a path (Sec. 2.4; App. C Eq. S19-S21): the Python
face of turpy_place_screens.  Host arithmetic in the library; no GPU needed.

    prof = placement.hufnagel_valley(A=1e-13)
    path = placement.placed_path(prof, length=3000.0, wavelength=1.064e-6, n=1024, dx=1e-3,
                                 rytov_limit=0.1, l0=0.005, L0=20.0, realizations=64)
"""

from dataclasses import dataclass
from typing import Optional, Tuple

from . import binding as B
from .workloads import Path


@dataclass(frozen=True)
class Cn2Profile:
    kind: int
    cn2: float = 0.0
    A: float = 0.0
    V: float = 0.0
    z: Optional[Tuple[float, ...]] = None
    values: Optional[Tuple[float, ...]] = None

    def descriptor(self):
        return B.make_cn2_profile(self.kind, self.cn2, self.A, self.V, self.z, self.values)


def uniform(cn2):
    """Constant Cn2 [m^-2/3]."""
    return Cn2Profile(B.CN2_UNIFORM, cn2=float(cn2))


def hufnagel_valley(A=1.7e-14, V=21.0):
    """Eq. S21 (z = height above the ground); the defaults are the HV 5/7 profile."""
    return Cn2Profile(B.CN2_HUFNAGEL_VALLEY, A=float(A), V=float(V))


def table(z, values):
    """Piecewise linear through (z[i], values[i]); constant beyond the ends."""
    return Cn2Profile(B.CN2_TABLE, z=tuple(float(x) for x in z), values=tuple(float(v) for v in values))


def place_screens(profile, length, wavelength, n, dx, rytov_limit, initial=1, n0=1.0):
    """Screen placement: {"dz": [M+1], "cn2dz": [M], "rytov": [M]} (see turpy_place_screens)."""
    dz, cn2dz, rytov = B.place_screens(profile.descriptor(), float(length), float(wavelength), float(n0), int(n),
                                       float(dx), float(rytov_limit), int(initial))
    return {"dz": dz, "cn2dz": cn2dz, "rytov": rytov}


def placed_path(profile, length, wavelength, n, dx, rytov_limit, initial=1, n0=1.0, **path_fields):
    """A Path whose screens come from place_screens; other Path fields by keyword."""
    res = place_screens(profile, length, wavelength, n, dx, rytov_limit, initial, n0)
    return Path(n=int(n), dx=float(dx), wavelength=float(wavelength), dz=tuple(res["dz"]),
                cn2dz=tuple(res["cn2dz"]), n0=float(n0), **path_fields)
