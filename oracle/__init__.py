"""MTGP oracle -- test infrastructure only.

Plain CPU implementations written from the paper, used to check the HIP
library. Only tests, the smoke check and the benchmark's CPU-baseline leg may
import anything from this package; the library never does.
"""
