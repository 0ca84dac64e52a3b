"""MI355X-native fluctuating lattice-Boltzmann hot path (D3Q19 MRT with
thermal noise and frictional point-particle coupling), after Duenweg & Ladd,
"Lattice Boltzmann simulations of soft matter systems".

The numerical work lives in liblbmi.so (HIP, gfx950) behind the C ABI of
include/lb.h; this package is the Python binding.
"""
from ._lib import LBError, load  # noqa: F401

__all__ = ["LBError", "load", "Lattice", "BatchLattice", "FluidParams", "DeviceBeads"]


def __getattr__(name):
    if name in ("Lattice", "BatchLattice", "FluidParams", "DeviceBeads"):
        from . import lattice
        return getattr(lattice, name)
    raise AttributeError(name)
