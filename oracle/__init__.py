"""CPU oracle for the Pauli decomposition -- test infrastructure only.

Imported by the tests, the smoke check and the benchmark (its CPU baseline,
and the errors it states against the oracle on sampled strings); never by
the product library.  See oracle.py and oracle.c.
"""
