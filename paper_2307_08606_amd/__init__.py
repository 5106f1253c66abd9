"""MI355X sharing-ADMM radar imaging engine (accelerated SADMM with pixel
elimination), behind the C ABI of include/sadmm.h.

`sadmm_lib` is the ctypes binding of libsadmm.so; build the library with
`python -m paper_2307_08606_amd.build`.
"""

__all__ = ["sadmm_lib"]
