"""CPU oracle for the pruned k-NN scan.

TEST INFRASTRUCTURE ONLY: this package is the independent checker.  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import,
call, link or execute anything under oracle/.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constants) and the library
never imports it.

  brute.py     O1/O2: brute-force exact k-NN (flat and IVF exact-at-probe)
               with the canonical distance recipe, in FP64.
  panorama.py  O3: a plain serial pruned scan (Algorithm 1) in FP64, the PCA
               fit (Section 4.1) and the bound quantities of Eq. 1-4.
  c/           the same O1/O2/O3 in plain C with OpenMP over queries, used to
               time the CPU baseline.
"""
