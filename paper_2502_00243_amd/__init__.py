"""FPW periodogram on AMD Instinct MI355X (gfx950).

The compute path is the HIP library ``libfpw.so`` (built from ``csrc/``);
``fpw`` is a thin ctypes binding over its C ABI.  Importing the binding
does not load the library; the first call does, and fails loudly when the
library is missing.
"""
