"""CPU oracle for GBS probabilities and hafnians -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. It shares no code with the GPU library: it computes B, gathers the
pattern matrices and evaluates hafnians itself, in plain double (or long double)
arithmetic on the CPU.
"""
from .oracle import *  # noqa: F401,F403
