"""FP64 CPU oracle for the GaBP SVM solver (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use this package.  The HIP library never imports or links it.
"""
