"""MI355X-native brute-force short-coherence statistic (arXiv:2411.18370 hot path).

The compute path lives in the HIP/C library ``libfasttracks.so`` (sources in
``csrc/``, C ABI in ``include/fasttracks.h``); ``fasttracks`` is its thin ctypes
binding and ``synth`` produces seeded synthetic inputs.  Importing this package
does not load the GPU library; ``paper_2411_18370_amd.fasttracks`` does.
"""
__all__ = ["synth", "fasttracks"]
