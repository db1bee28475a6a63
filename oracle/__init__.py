"""CPU oracle (FP64 NumPy) for masked LDDMM -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py may
import this package; the product path never does.
"""
