"""CPU oracle of the fault-tolerant GEMM -- test infrastructure only.

Loaded by the tests, the smoke check and the benchmark's CPU-baseline leg;
the product library never imports anything from here.
"""
