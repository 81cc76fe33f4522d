"""CPU oracle for SimpleX2 DCT transport + hydrogen chemistry.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.
"""
from .oracle import Oracle, build_oracle, chem_cell, oracle_lib_path  # noqa: F401
