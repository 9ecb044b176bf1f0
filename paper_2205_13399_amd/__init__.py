"""MI355X multi-objective Digital Annealer (arXiv:2205.13399) on the bi-objective QAP.

The annealing path is HIP code in ``libmda.so`` behind the C ABI of
``include/mda.h``; ``paper_2205_13399_amd.mda`` is its Python binding.
"""
__all__ = ["mda"]
