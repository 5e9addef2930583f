"""Block-sparse x dense matmul (PopSparse, arXiv 2303.16999) on AMD MI355X (gfx950).

The compute runs in hand-written HIP kernels behind a C ABI (include/spmm.h);
`paper_2303_16999_amd.spmm` is the thin ctypes binding. Importing this package
does not load the library; `spmm.lib()` does, and fails loudly if it is missing.
"""
