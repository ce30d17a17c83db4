"""Windowed KSG mutual information on AMD MI355X (gfx950).

The GPU library ``libwmi.so`` (HIP kernels + C-ABI runtime, sources in
``csrc/``) is reached through the thin ctypes binding in ``wmi.py``; import it
explicitly (``from paper_2204_09131_amd import wmi``).  ``synth`` holds the
seeded input generators and none of the estimator's arithmetic.
"""
__all__ = ["synth", "wmi"]
