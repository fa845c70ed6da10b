"""Plain FP64 CPU oracle for the directional wavelet transform on the sphere
and the ball (Price, Polanska, Whitney & McEwen, "Differentiable and
accelerated directional wavelet transforms on the sphere and ball").

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__
and the CPU-baseline leg of bench.py may import, call, link or execute
anything under oracle/.  The product path (paper_2402_01282_amd/) never
does, and the two share no code.

Layout of the oracle:
  wigner_oracle.c  Delta = d(pi/2) tables, Fourier-space Wigner sums,
                   Wigner's explicit sum (C, long double / double, OpenMP)
  mw.py            McEwen-Wiaux sampling, exact theta quadrature,
                   spherical-harmonic and Wigner transforms and their adjoints
  filters.py       scale-discretised tiling functions and wavelet filters
                   (paper Appendix A)
  wavelets.py      sphere analysis / synthesis / adjoint (paper Section 4,
                   Algorithm 1)
  ball.py          Laguerre radial transform and ball wavelets (paper
                   Section 5, Algorithm 2)

Every function cites the passage of the paper it follows.  Readings of
passages that are silent or garbled are stated where they are used.
"""
from . import _lib  # noqa: F401
