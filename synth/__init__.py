"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the energy model. It only draws inputs:
liquid-ammonia-shaped atom positions, Maxwell-Boltzmann velocities and flat
weight blobs of standard normals scaled by 1/sqrt(fan_in). The weight blob's
segment shapes are passed in by the caller; both the oracle and the GPU library
state their own segment order, and a test checks that the two agree.
"""
from .configs import CONFIGS, ModelDesc, SystemSpec, config
from .nh3 import make_system, maxwell_boltzmann
from .weights import weight_blob

__all__ = ["CONFIGS", "ModelDesc", "SystemSpec", "config", "make_system",
           "maxwell_boltzmann", "weight_blob"]
