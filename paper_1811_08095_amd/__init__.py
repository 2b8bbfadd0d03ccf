"""MI355X-native even-odd optimal domain-wall fermion operator and CG solves.

The compute path is the HIP library libodwf.so (csrc/); this package holds its
thin ctypes binding (odwf.py), the serving loop (serve.py) and the seeded
synthetic-input generator (synth.py).  Importing the package loads nothing; the
library is opened on first use and raises if it has not been built.
"""
