"""MI355X (gfx950) implementation of the TTCF daughter path of arxiv 2312.02990.

The computation lives in libttcf.so (HIP kernels behind the C ABI of include/ttcf.h);
``paper_2312_02990_amd.ttcf`` is its Python binding.
"""
