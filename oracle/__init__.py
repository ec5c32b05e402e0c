"""Plain CPU oracle for randomized block matrix multiplication by sampling.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code, table or
constant generator with the HIP library in ``paper_2105_04940_amd``, and it
never imports that package.

Everything here is float64 NumPy or pure-Python integers, written from the
paper (Niu & Li, "Optimal Sampling Algorithms for Block Matrix
Multiplication", arXiv 2105.04940) and, for the random-number generator, from
Salmon et al., "Parallel random numbers: as easy as 1, 2, 3" (SC'11).

Modules
-------
rng       Philox4x64-10 and the counter layout used to draw sample indices.
sampling  Integer weight quantization, per-stratum CDF, Lemire's exact
          bounded integer, CDF search and the integer draw-count allocation.
method    The estimator itself: norms, design rules (1.1)-(1.4), (3.8), (3.9),
          (4.2), Alg. 1 / Alg. 2 sampling, the pilot and block sizes (4.7)
          of the two-step Alg. 3, the sketch C, D, the product CD, the judge
          ||MN - CD||_F, the closed-form expected error (Thm 2 proof /
          Remark 2.2) and the gradient of the sketch.
lowp      bfloat16, E4M3 and the MX block format (reduced-precision sketches).

Pins: every function is checked in ``tests/test_oracle_*.py`` against values
fixed by the paper or by mathematics (known-answer vectors, exhaustive
enumeration, closed forms, library routines, special cases). A function with
no such pin says "parity unpinned" in its docstring; there are none at
present.
"""

from . import rng, sampling, method  # noqa: F401
