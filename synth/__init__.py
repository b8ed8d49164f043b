"""Seeded synthetic input generators shared by the tests and the benchmark."""
from .philox import philox4x32, element_words  # noqa: F401
from . import workloads  # noqa: F401
