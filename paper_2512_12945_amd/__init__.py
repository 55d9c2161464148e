"""MI355X-native fused TSDF + Bayesian semantic integration (SLIM-VDB, arXiv 2512.12945).

The compute path is the HIP library ``libslimvdb.so`` behind a C ABI
(``include/slimvdb.h``); ``paper_2512_12945_amd.slimvdb`` is its thin Python
binding.  ``paper_2512_12945_amd.synth`` generates seeded synthetic inputs.
Importing this package loads nothing; the library is loaded on first use.
"""
__all__ = ["slimvdb", "synth"]
