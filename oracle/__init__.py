"""CPU oracle (test infrastructure only): plain complex128 state-vector
reference and a brute-force Kronecker checker.  Imported only by the tests,
the smoke check and the benchmark's CPU-baseline leg."""
