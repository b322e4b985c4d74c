"""MI355X (gfx950) library for the moment-matching lattice Boltzmann scheme
for warm relativistic plasma wakes of Simeoni et al. (arXiv 2309.04872).

The hot path is hand-written HIP (``csrc/``) behind the C ABI of
``include/lbwake.h``; ``Sim`` is a thin ctypes binding over it. Importing the
package does not load the library; constructing a ``Sim`` does, and fails
loudly when ``liblbwake.so`` has not been built.
"""
from ._lib import LibraryMissing  # noqa: F401


def __getattr__(name):
    if name in ("Sim", "LbwError"):
        from . import sim

        return getattr(sim, name)
    raise AttributeError(name)
