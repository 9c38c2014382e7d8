"""CPU FP64 reference for exact Reverse k-MIPS -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (the HIP library and its Python binding) never does.
"""
