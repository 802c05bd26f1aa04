"""MI355X-native D2Q9 MRT lattice-Boltzmann step with the curved slip boundary of
Wang et al. (arXiv:2012.14707).

Submodules:
  geometry  seeded problem generators (masks and wall-link tables); no lattice arithmetic
  lbm       ctypes binding of the HIP library ``liblbm.so`` (loaded on first use)
"""
__all__ = ["geometry", "lbm"]


def __getattr__(name):
    if name in ("lbm", "geometry"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
