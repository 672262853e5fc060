"""FP64 CPU oracle for the splatting and decoding path (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package. The product library never does.
"""
