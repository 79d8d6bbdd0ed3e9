"""MI355X-native coupled LBM-PSM-DEM time step (arXiv 2512.04997).

The compute path is the HIP library ``libpsmdem.so`` (C ABI declared in
``include/psmdem.h``); :mod:`paper_2512_04997_amd.psmdem` is its thin ctypes
binding and :mod:`paper_2512_04997_amd.workloads` the seeded synthetic inputs.
Importing the package loads nothing native; the binding loads the library on
first use and raises if it is missing.
"""
__all__ = ["psmdem", "workloads"]
