"""CPU oracle for the Cartesian FMM of point dipoles (test infrastructure only).

This package is the plain FP64 reference the GPU library is checked against:
an O(N^2) brute-force dipole sum and the paper's recursive Cartesian FMM
(three recursive passes over a pointer tree, Sec. 2 and Appendix).  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the GPU library (``paper_0810_0233_amd``)
and never imports it.
"""
from .ccref import *  # noqa: F401,F403
