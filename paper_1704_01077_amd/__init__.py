"""Exact top-k closeness centrality on AMD Instinct MI355X (gfx950).

The work runs in the HIP library ``libtkc.so`` (sources in ``csrc/``, C ABI
in ``include/tkc.h``); ``paper_1704_01077_amd.tkc`` is its Python binding.
Importing the binding fails loudly when the library has not been built.
"""
