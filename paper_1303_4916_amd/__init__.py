"""MI355X-native electron-repulsion integrals and Coulomb/exchange (Fock) builds.

The compute path is the HIP library ``libuqc.so`` (C ABI in include/uqc.h); ``uqc`` is its Python binding and
``workloads`` the seeded synthetic input generator.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "uqc"]
