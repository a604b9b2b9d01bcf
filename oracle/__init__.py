"""Plain FP64 CPU oracle of the per-particle ADM1 reaction step.

TEST INFRASTRUCTURE ONLY: used by the tests, the package smoke check and the
CPU-baseline leg of the benchmark; never by the product path.
"""
