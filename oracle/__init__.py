"""CPU reference for noise-canceling Pauli propagation (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the HIP library it checks.
"""
