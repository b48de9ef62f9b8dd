"""CPU oracle of the GZ1 codec and of the selector network.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  The C part
(gzo.c) is the codec; mlp.py holds the float64 training math of the selector.
"""
from .gzo import *  # noqa: F401,F403
