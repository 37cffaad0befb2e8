"""MI355X-native FIRLS: the PCG hot path of analysis-sparsity CS-MRI
reconstruction as hand-written HIP kernels for gfx950 behind a C ABI.

``paper_1411_5057_amd.firls`` is the ctypes binding of ``libfirls.so``
(declared in ``include/firls.h``); ``paper_1411_5057_amd.build`` compiles it.
Importing this package loads nothing; the binding loads the library on
first use and raises if it has not been built.
"""
