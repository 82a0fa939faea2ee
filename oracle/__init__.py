"""CPU oracle for the SPDZ online-phase arithmetic -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import or run anything in this package; the device library
never does.  It shares no code with the device path.

Two tiers, both written from the protocol's definitions:
  * `oracle.ref`  -- Python integers, for small inputs and exhaustive checks;
  * `oracle.fast` -- the same definitions in plain C (spdz_oracle.c) with
    128-bit integers and Knuth long division, for full-size workloads.
"""
