"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  Patterns and values only: none of the method's arithmetic."""
from . import patterns, values  # noqa: F401
from .configs import get_config, CONFIG_NAMES  # noqa: F401
