"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package generates signals, their noise-free components and their true
instantaneous frequencies.  It holds none of the transform's arithmetic: no
window, no DFT, no reassignment, no reconstruction.
"""
from .signals import (  # noqa: F401
    Workload,
    SSTConfig,
    make_c1,
    make_c2,
    make_c3,
    make_c4,
    make_c5,
    make_paper_eq30,
    make_tone,
    make_chirp,
    ridge_bins,
)
