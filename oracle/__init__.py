"""FP64 CPU oracle of the additive overlapping DDM (Leng & Ju, arXiv 1807.04180).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library (paper_1807_04180_amd); both are fed by the seeded input
generators in ddm_inputs, which hold none of the method's arithmetic.

Every function here is pinned by tests in tests/test_oracle_*.py to something
other than itself (closed forms, a dense library solve, invariants of the
method); see the module docstrings there.
"""
from .oracle import Oracle, build_oracle  # noqa: F401
