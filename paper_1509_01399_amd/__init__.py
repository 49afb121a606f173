"""MI355X-native domain-decomposition FEM/FDM wave solver (arXiv 1509.01399).

The compute path lives in the HIP library ``libhyb.so`` (built from
``csrc/``); ``hyb`` is its thin ctypes binding.  Importing this package does
not load the library: ``paper_1509_01399_amd.hyb`` loads it on first use and
raises if it is missing.
"""
__all__ = ["synth"]
