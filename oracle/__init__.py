"""FP64 CPU oracle for the root-coupled branch system (TEST INFRASTRUCTURE).

Imported only by the tests, the smoke check and the benchmark's CPU-baseline leg;
the product library never uses it.
"""
