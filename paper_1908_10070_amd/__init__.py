"""MI355X-native batched GBS probabilities and hafnians (arXiv:1908.10070 hot path).

The compute path is the HIP library ``libgbs.so`` (C ABI, ``include/gbs.h``);
``paper_1908_10070_amd.gbs`` is its thin Python binding. Importing this package
does not load the library; ``inputs`` (seeded synthetic workloads) needs numpy only.
"""
__all__ = ["gbs", "inputs", "serve", "autotune"]
