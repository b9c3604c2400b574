"""MI355X (gfx950) Schroedinger-Feynman path-sum library (arXiv:1807.10749).

The product is libsfpath.so (C ABI in include/sfpath.h); ``binding`` is its
ctypes binding.  Importing the package does not load the library, so host
tools can import it on machines without the build; importing
``paper_1807_10749_amd.binding`` does, and raises if it is missing.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsfpath.so")
