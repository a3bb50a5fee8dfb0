"""orng: counter-based random number generation for MI355X (gfx950).

The compute path is the HIP library ``liborng.so`` (C-ABI, ``include/orng.h``);
``paper_2310_19925_amd.orng`` is its thin ctypes binding.  Importing this package
does not load the library; the binding loads it on first use and raises if it
is missing.
"""
__all__ = ["orng", "inputs"]
