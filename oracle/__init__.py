"""Plain FP64 CPU oracle for the Khatri-Rao random projection (KRP) methods.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, constants or
helpers with the HIP implementation in ``paper_2507_23207_amd``; the only code
both sides use is the seeded input generator package ``synth``, which holds
none of the method's arithmetic.

Everything here is written for a reader holding the paper (Saibaba, Verma,
Ballard, "Improved Analysis of Khatri-Rao Random Projections and
Applications"): every product is formed explicitly (Khatri-Rao products,
unfoldings, the block-Hankel matrix), in float64, with LAPACK/BLAS through
numpy for the dense matrix primitives.

Modules
-------
rng      Philox4x64-10 counter generator and the Box-Muller Gaussian transform
         (the random factors of Definition 2.1).
tensor   Unfolding, TTM, Khatri-Rao products and the explicit MTTKRP sketch.
linalg   Thin QR with a positive-diagonal R.
tucker   Algorithms 4, 5, 7 and 8 plus truncation and Tucker errors.
hankel   Algorithm 6 specialised to block-Hankel matrices (Section 4.2).
counts   Random-number counts of Table 1 and Section 4.1.
"""
