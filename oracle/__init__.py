"""The oracle: a plain, slow, obviously correct CPU implementation of LTL4-C
monitoring, written from the paper (arXiv 1411.2239) and pinned by tests.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import, call or link anything in this package.  It
shares no code with the product library (paper_1411_2239_amd) and imports
nothing from it; the product library never imports it.

  oracle.ltl       FLTL (Def. 4), LTL4 (Def. 5) via an atom tableau, and a
                   monitor built from that semantic state (Def. 6)
  oracle.counting  value vectors, clusters and the counting semantics
                   (Eq. 5-6, Def. 7, Table 1, Def. 8) in Python
  oracle.cref      the plain C evaluator (oracle/c/ltl4c_oracle.c) used for
                   full-size parity checks and the timed CPU baseline
"""
