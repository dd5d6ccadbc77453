"""libftgemm: fault-tolerant GEMM (ABFT fused into the GEMM) for AMD MI355X.

The compute path is the HIP library ``libftgemm.so`` built from ``csrc/``;
``ftgemm`` is its thin ctypes binding.  ``synth`` draws the seeded synthetic
workloads.
"""
