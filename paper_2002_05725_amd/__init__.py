"""MI355X (gfx950) implementation of the matrix-free SYK hot path of
arXiv:2002.05725: H|psi> for the Jordan-Wigner q=4 SYK Hamiltonian, Krylov
propagation, two-point functions and regularized OTOCs from typical states.

The computation lives in the HIP library libsyk.so (C interface:
include/syk.h); ``api`` binds it for torch GPU tensors.  ``inputs`` draws
the seeded synthetic couplings and states.  Importing the package loads
nothing; the library is loaded on the first call.
"""
__version__ = "0.1.0"


def __getattr__(name):
    if name in ("api", "inputs", "build"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    from . import api
    if hasattr(api, name):
        return getattr(api, name)
    raise AttributeError(name)
