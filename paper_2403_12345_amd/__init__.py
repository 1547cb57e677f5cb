"""MI355X-native hot path of event-based continuous-energy Monte Carlo
neutral-particle transport (HIP kernels for gfx950 behind the C ABI of
include/mc.h).

``paper_2403_12345_amd.mc`` is the ctypes binding (same names as the C entry
points); ``paper_2403_12345_amd.transport`` fills the library's structs from a
problem description.  Importing this package does not load the library;
calling an entry point does, and raises if libmc.so has not been built.
"""
from . import mc  # noqa: F401
from .build import build_library, library_path  # noqa: F401
