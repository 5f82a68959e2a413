"""CPU oracle for the ray-tracing radiative-transfer hot path.

TEST INFRASTRUCTURE ONLY.  The plain FP64 reference the HIP library is checked
against.  Only tests, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the HIP library (`paper_2011_14998_amd`),
and the product never imports it.
"""
from .oracle import *  # noqa: F401,F403
