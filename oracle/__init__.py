"""Reference implementations of closed-form 3x3 eigenvalues (arXiv 2511.00292).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything in this package.  It shares no code with the HIP library in
``paper_2511_00292_amd`` and never imports it.

* ``oracle.exact``  -- the definitions (invariants, characteristic-polynomial
  roots, eigenprojector gradient, stability-bound scales) in exact rational /
  80-digit arithmetic: the truth every forward error is measured against.
* ``oracle.plain``  -- the paper's algorithms (Alg. alg:I1-stable,
  alg:J2-stable, alg:J3-stable, alg:disc-stable, alg:eigvals-stable) in plain
  binary64 C without FMA (``eig3_plain.c``), plus an eigenprojector-based
  backward; the timed CPU baseline and the "paper's own algorithm" allowance.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, constructed spectra, independent definitions and the
paper's worked example; none is "parity unpinned".
"""
