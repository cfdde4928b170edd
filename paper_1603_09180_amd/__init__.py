"""MI355X lambda-leveling (Couprie-Bertrand grayscale thinning) library.

The compute path is the HIP library libthin.so (include/thin.h); thin.py is
its ctypes binding.  Importing the package does not load the library, so the
input generators (synth) stay usable on machines without a GPU; every call
into the binding fails loudly when the library is missing.
"""
from .thin import (  # noqa: F401
    Context,
    Stats,
    ThinError,
    load_library,
    run,
)
