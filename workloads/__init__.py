"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds random-number draws and closed-form initial fields only --
none of the scheme's arithmetic -- so that the oracle and the HIP path can be
fed bit-identical inputs without sharing any code of the method.
"""
from .synth import (Instance, WORKLOADS, batched_instances, cosine_mode, paper_ic_51,
                    smooth_ic_2d, uniform_field)

__all__ = ["Instance", "WORKLOADS", "batched_instances", "cosine_mode", "paper_ic_51",
           "smooth_ic_2d", "uniform_field"]
