"""FDAS hot path on AMD Instinct MI355X (gfx950).

``fdas``     ctypes binding of libfdas.so (plan, templates, correlate, peaks)
``metrics``  the paper's plane measurements (Eq. 2, SNR, Table 3 bands, bin match)
``build``    in-tree hipcc build of libfdas.so

Importing the package loads nothing; the library is loaded on first use and
its absence is an error.
"""
__all__ = ["fdas", "metrics"]
