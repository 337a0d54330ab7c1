"""Seeded synthetic LP workloads shared by the reference solver and the GPU library."""
from .generators import *  # noqa: F401,F403
