"""MI355X-native engine for the USApHMP parallel genetic algorithm (arXiv 1704.06258).

The compute path is ``libhubga.so`` (hand-written HIP kernels for gfx950 behind
the C ABI declared in ``include/hubga.h``); ``hubga`` is its ctypes binding.
Importing this package does not load the library; ``hubga.lib()`` does.
"""
