"""Minimum enclosing ball of balls on MI355X: mixed-precision ripALM.

The compute path is the HIP library ``libmeb.so`` (built from ``csrc/``),
reached through the thin ctypes binding in ``meb.py``.  ``inputs.py`` holds
the seeded synthetic instance generators.  Importing this package loads
nothing; ``paper_2605_31425_amd.meb`` loads the library on first use.
"""
