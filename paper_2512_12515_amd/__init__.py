"""MI355X-native density-fitted particle-particle RPA (ppRPA) hot path.

The compute runs in libpprpa.so (HIP kernels for gfx950 behind the C ABI of include/pprpa.h);
this package only builds and binds it.
"""
from .binding import PpRPA, PpRPAError, Server, lib, pprpa_build, pprpa_davidson, pprpa_free, pprpa_matvec  # noqa: F401
