"""MI355X (gfx950) implementation of the hot path of the seamless heterogeneous
multiscale method (Lee & Engquist, arXiv:1510.00451) behind a C ABI.

``abi`` is the thin ctypes binding of libshmm.so (names as in include/shmm.h);
``hierarchy`` drives the phases of one pass through the library's entry points.
Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing (there is no CPU fallback).
"""
