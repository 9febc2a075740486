"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only draws random matrices with prescribed singular spectra and
builds the snapshot-shaped stand-in workload.  It contains none of the
interpolative-decomposition arithmetic (no pivoting, no reflectors, no solves);
both the CPU oracle and the HIP path consume what it returns.
"""
from .inputs import *  # noqa: F401,F403
