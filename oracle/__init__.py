"""Plain FP64 CPU oracle of the scattered-field PIC step (1D, 2D and 3D).

TEST INFRASTRUCTURE ONLY: imported by tests/, the package smoke check and the
benchmark's CPU-baseline leg.  The product path never imports it.
"""
from .oracle import OracleSim, OracleSim3, april_complex, incident_eval, \
    incident_eval3, shape2, boris, ka_from_w0, incident_norm  # noqa: F401
