"""MI355X-native orthogonalization-free spectral clustering (OFM / TriOFM).

Importing the package loads nothing compiled; ``paper_2305_10356_amd.ofm``
loads the HIP library on first use and fails loudly if it is missing.
"""
__all__ = ["graphs"]
