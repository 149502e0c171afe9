"""CPU oracle for the irradiance-matrix hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations written from the
paper (arXiv 2103.14137, Sec. III-B and Sec. IV-C/D): FP64 brute-force
irradiance and visibility (uvc_oracle.c), an exact rational segment/triangle
predicate (exact.py), the relaxed dosage LP through SciPy's HiGHS (lp.py) and
FP64 references of the ranker's features, MLP, loss and Adam step
(ranker.py).  Only tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py may import anything from this package; the
product path (paper_2103_14137_amd) never does.
"""
