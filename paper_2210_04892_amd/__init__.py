"""MI355X library for the MLFMA-accelerated boundary-integral matrix-vector
product of the coupled HDG-BI method (arXiv 2210.04892).

The C ABI is declared in include/mlfma.h; `binding` is its thin Python
binding (torch provides device memory and streams)."""
from .binding import (Geometry, Graph, Server, Hybrid, MlfmaError, translation_operator, matvec_batch, peak_probe, OP_C,
                      OP_EM, C128, C64, LIB_PATH, PART_NEAR, PART_FAR, PART_ALL, PART_LEVEL)

__all__ = ["Geometry", "Graph", "Server", "Hybrid", "MlfmaError", "translation_operator", "matvec_batch", "peak_probe", "OP_C",
           "OP_EM", "C128", "C64", "LIB_PATH", "PART_NEAR", "PART_FAR", "PART_ALL", "PART_LEVEL"]
