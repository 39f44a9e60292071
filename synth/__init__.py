"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

Holds random draws and gate lists only; none of the simulation arithmetic."""
from .circuits import *  # noqa: F401,F403
