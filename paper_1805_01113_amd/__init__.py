"""MI355X-native moving-least-squares immersed-boundary transfer (arXiv:1805.01113).

The compute path lives in the HIP library ``libmls_hip.so`` (C ABI declared
in ``include/mls.h``); :mod:`paper_1805_01113_amd.mls` is its thin Python
binding and :mod:`paper_1805_01113_amd.workloads` generates seeded inputs.
Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__version__ = "0.1.0"
