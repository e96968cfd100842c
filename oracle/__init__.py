"""CPU oracle for the BI matrix-vector product (test infrastructure only).

Only tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library.
"""
from .oracle import (build, rwg_table, matvec, pair_integrals, pair_integrals_sub, leaf_boxes, class_box_pairs, threads,
                     plane_wave_rhs, far_field, entries, blocks, OP_C, OP_EM, OP_BOTH, PRIM)
from . import sai

__all__ = ["build", "rwg_table", "matvec", "pair_integrals", "pair_integrals_sub", "leaf_boxes", "class_box_pairs", "threads",
           "plane_wave_rhs", "far_field", "entries", "blocks", "sai", "OP_C", "OP_EM", "OP_BOTH", "PRIM"]
