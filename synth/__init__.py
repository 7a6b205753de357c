"""Seeded synthetic particle sets shared by the tests, the smoke check and the bench.

This package only draws inputs (positions, smoothing lengths, masses, targets'
perturbations). It holds no part of the density computation: neither the kernel
function nor any neighbour sum. The one geometric check it performs -- rejecting
inputs that have a particle pair within a relative 1e-5 of a receiver's cut-off --
uses scipy's k-d tree as a plain distance-counting primitive.
"""
from .generators import *  # noqa: F401,F403
