"""CPU oracle for the implicit 2D3V PIC particle stage -- TEST INFRASTRUCTURE ONLY.

A plain FP64 C implementation (``orc.c``) of what the particle stage computes, plus a small
Python driver that holds the state in numpy arrays and calls the C functions in the order of
one PIC cycle.  Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline may import it; the GPU library never does, and this package never imports the GPU
library.
"""
from .oracle import OracleSim, build, load_library  # noqa: F401
