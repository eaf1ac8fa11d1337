"""MI355X row-wise hash SpGEMM (SMASH, arXiv 2105.14156).

Importing the package loads nothing; ``paper_2105_14156_amd.smash`` binds the
HIP library (``libsmash.so``) and raises if it has not been built.
"""
