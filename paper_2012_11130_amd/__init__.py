"""MI355X (gfx950) SRHD patch-step library after Tseng, Schive & Chiueh, arXiv:2012.11130.

The compute path is libsrhd.so (HIP kernels behind the C ABI of include/srhd.h); ``srhd`` is its
ctypes binding.  Build with ``python -m paper_2012_11130_amd.build``.
"""
