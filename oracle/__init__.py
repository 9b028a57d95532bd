"""CPU oracle for the QCT hot path -- TEST INFRASTRUCTURE ONLY.

A plain serial FP64 implementation of the method of Koots & Perez-Rios,
arXiv:2304.02731, written independently of the HIP library.  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import it.
"""
from .oracle import *  # noqa: F401,F403
