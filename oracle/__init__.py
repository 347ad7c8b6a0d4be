"""CPU oracle package.  TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke
check and the benchmark's CPU-baseline leg, never by the product path."""
