"""FP64 CPU oracle for block-sparse x dense matmul (PopSparse, arXiv 2303.16999).

TEST INFRASTRUCTURE ONLY. Nothing in the library imports this package. Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import or
call it. It shares no code with the HIP path: it is written from the paper's
definition (Section 3) in plain NumPy float64, slowly and obviously.

Modules
-------
spmm_ref  the SpMM definition Y = (M o W) * X three ways (expand, brute force,
          blockwise), the relative Frobenius error and the useful-FLOP count.
fp8_ref   decoding of OCP E4M3FN codes from the format definition, and per-block
          dequantisation (code value times FP32 block scale) in float64.
plan_ref  the static plan (block-CSR, row groups, cost-balanced panels, in-group
          column-major order) derived with NumPy primitives, plus a pure-Python
          loop version for tiny inputs.
"""
