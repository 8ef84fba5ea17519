"""Minimum-initial-credit solver for energy games on MI355X (gfx950).

The solver itself is the C-ABI library ``libeg.so`` built from ``csrc/``; the
Python module ``eg`` marshals arguments to it.  ``synth`` draws seeded inputs.
Importing the package loads nothing.
"""
