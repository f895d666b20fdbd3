"""Plain FP64 CPU oracle for the local-f_NL map generator.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP library; see fnl_oracle.c for what it computes.
"""
