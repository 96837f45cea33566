"""MI355X-native batched gradient of forward dynamics (GRiD, arXiv 2109.06976).

Importing the package loads nothing native; `paper_2109_06976_amd.grid` holds the
binding to the HIP library.
"""
