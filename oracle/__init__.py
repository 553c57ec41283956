"""FP64 CPU oracle of the preconditioned NCG-MLS field-map estimator.

Test infrastructure only: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.
"""
from .oracle import *  # noqa: F401,F403
