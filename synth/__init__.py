"""Seeded synthetic workloads shared by the GPU path's tests/benchmark and the oracle.

This package only draws random numbers and shapes them into signals, impulse
responses and switching schedules. It holds none of the convolution method's
arithmetic, so both sides can take their inputs from it without sharing any
part of the computation under test.
"""
from .workloads import *  # noqa: F401,F403
