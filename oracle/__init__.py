"""TEST INFRASTRUCTURE ONLY: the plain fp64 CPU oracle of the MSP connectivity update.

Imported only by the tests, the smoke check and the benchmark's CPU-baseline leg.
"""
