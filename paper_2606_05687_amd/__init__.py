"""MI355X-native batched parallel-in-horizon MPC solver (pi^n MPC hot path).

The solver is the HIP library libpinmpc.so (C ABI in include/pinmpc.h);
``binding`` marshals torch device tensors into it.  Importing the package does
not load the library; ``binding.load()`` (or constructing a ``Solver``) does,
and raises if it was not built.
"""
from .binding import Solver, default_settings, load, to_device  # noqa: F401
