"""In-situ reduction of spectral-element snapshots on MI355X (gfx950).

The product path is the HIP library ``libisr.so`` (C ABI in include/isr.h);
``paper_2407_20731_amd.isr`` is its Python binding.  Import the binding
explicitly: ``from paper_2407_20731_amd import isr``.
"""
