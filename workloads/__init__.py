"""Seeded synthetic inputs shared by the CPU oracle and the HIP path."""
from .configs import *  # noqa: F401,F403
