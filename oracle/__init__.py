"""CPU oracle: plain FP64 reference of QR- and EVD-based C3v CTMRG on the
honeycomb lattice (arXiv 2509.05090).  TEST INFRASTRUCTURE ONLY: imported by
tests, the smoke check and the benchmark's CPU-baseline leg, never by the
product library."""
