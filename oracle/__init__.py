"""CPU oracle for the KFAC-PINN hot path (FP64, plain PyTorch on the CPU).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product path (the HIP library and its Python
binding) never imports, calls or links anything here.
"""
from .kfac import *  # noqa: F401,F403
from . import kfac  # noqa: F401
