"""MI355X-native ternary colour-gradient lattice Boltzmann step (arXiv:1808.08555).

Importing the package loads nothing; ``paper_1808_08555_amd.lbm3`` is the binding
to the HIP library ``liblbm3.so`` and ``paper_1808_08555_amd.inputs`` holds the
seeded synthetic input recipes.
"""
__all__ = ["inputs", "lbm3"]
