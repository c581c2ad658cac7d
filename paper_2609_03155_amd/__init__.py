"""MI355X-native DPG local solve for the ultraweak time-harmonic Maxwell system.

The compute path is the HIP library ``libdpgmi.so`` (C ABI declared in
``include/dpg.h``); ``paper_2609_03155_amd.dpg`` is a thin ctypes binding with
the same entry-point names.  Importing this package does not load the
library; the binding loads it on first use and raises if it is missing.
"""
__all__ = ["dpg", "workloads"]
