"""CPU oracle for the BLDTT compute phase (test infrastructure only).

`oracle.core` wraps the plain C FP64 implementation; `oracle.brute` holds
independent NumPy brute-force forms for tiny inputs.  Nothing in the HIP
library imports this package.
"""
