"""MI355X-native round-synchronous innermost term rewriting.

``paper_2009_07174_amd.trs`` is the binding of the HIP library libtrs.so
(include/trs.h); ``paper_2009_07174_amd.build`` compiles it for gfx950.
"""
