"""CPU oracle for the SRK PT flash -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The library under ``paper_2205_03090_amd`` never does.
"""
from .oracle import *  # noqa: F401,F403
