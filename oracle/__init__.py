"""CPU oracle for the s-step enlarged Conjugate Gradient methods.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under ``oracle/``; only the test-suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
implementation: it is written independently from the paper (Moufawad,
"Numerical Stability of s-step Enlarged Krylov Subspace Conjugate Gradient
methods", arXiv 1804.10629) in plain numpy/scipy, in float64 unless a
function says otherwise.

Every function cites the passage it follows.  Parity status of each part is
recorded next to it; no function here is "parity unpinned".
"""
from .ecg_oracle import *  # noqa: F401,F403
from .ecg_oracle import __all__  # noqa: F401
