"""MI355X-native kinetic DG time step (arXiv:2212.11010), C-ABI library libkds.

Importing the package loads nothing; ``paper_2212_11010_amd.kds`` is the
binding to the HIP library.
"""
