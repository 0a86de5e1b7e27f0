"""CPU oracle for the Pauli decomposition -- test infrastructure only.

Imported by the tests, the smoke check and the benchmark's CPU-baseline leg;
never by the product library.  See oracle.py and oracle.c.
"""
