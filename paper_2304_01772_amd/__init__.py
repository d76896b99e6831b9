"""spinmc for MI355X: batched checkerboard Metropolis-Hastings sampling of
Ising, q-state Potts and Cellular Potts lattices (after "A differentiable
programming framework for spin models"), hand-written HIP for gfx950 behind
the C ABI in include/spinmc.h.

Importing the package does not load the library; ``Sampler`` does, and
raises if ``libspinmc.so`` has not been built.
"""
from ._lib import ISING, POTTS, CPM, SpinmcError  # noqa: F401


def __getattr__(name):
    if name == "Sampler":
        from .sampler import Sampler
        return Sampler
    raise AttributeError(name)
