"""FP64 CPU oracle of the constraint-penalization LBM step.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline
leg of bench.py.  The GPU library never imports, links or calls it.
"""
