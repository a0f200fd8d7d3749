"""MI355X (gfx950) linearized ordinary state-based peridynamics.

The solver lives in libpd.so (HIP kernels + host C++ behind the C ABI of
include/pd.h); this package holds its sources (csrc/), the build script and
a ctypes binding.  Importing the binding does not load the library; the
first call that needs it raises if libpd.so has not been built.
"""

from ._abi import load, PDError  # noqa: F401


def __getattr__(name):
    # the torch-based binding is imported lazily
    if name in ("Solver", "FamilyHost", "Context", "critical_stretch", "specimen_params"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
