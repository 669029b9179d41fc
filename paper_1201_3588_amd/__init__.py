"""MI355X-native Monte Carlo dust radiative transfer with transiently heated
PAHs (Siebenmorgen, Heymann & Kruegel).  The engine is libmcrt.so (HIP
kernels for gfx950 behind the C ABI of include/mcrt.h); ``mcrt`` and ``pah``
are its thin Python bindings.  Submodules load the library on first use.
"""
