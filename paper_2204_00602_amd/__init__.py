"""MI355X-native SLOS strong simulation (arXiv 2204.00602, Section 3.2.3).

Importing the package loads nothing native; the HIP library is loaded on the
first call that needs it and raises if it is missing.
"""
__all__ = ["inputs", "slos"]
