"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's
callers.  Holds no uplifting or diffusion arithmetic."""
from . import philox, scenes  # noqa: F401
