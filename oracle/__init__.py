"""FP64 CPU oracle for ViPer NL-COMM VP precoding.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.
"""
