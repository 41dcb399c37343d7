"""Two-stage dense symmetric eigenvalue decomposition for AMD MI355X (gfx950).

The compute path lives in the HIP library ``libevd.so`` (sources in
``csrc/``, C ABI in ``include/evd.h``); :mod:`.evd` is a thin ctypes binding
with the same entry-point names.
"""
