"""MI355X-native LTL4-C runtime verification (arXiv 1411.2239).

The hot path -- classifying events, grouping them by quantifier binding with a
stable radix sort, stepping every instance's LTL4 monitor with a segmented scan
of transition maps, and reducing the verdicts through the counting quantifiers
-- runs in hand-written HIP kernels for gfx950 behind the C ABI declared in
include/ltl4c.h.  This package holds the Python binding of that ABI
(`paper_1411_2239_amd.lib`), the LTL-to-LTL4-monitor compiler that produces the
transition tables the ABI consumes (`paper_1411_2239_amd.monitor`) and the
seeded workload generators (`paper_1411_2239_amd.workloads`).

Importing the package loads nothing; `lib.load()` opens the HIP library and
fails loudly if it has not been built.
"""
