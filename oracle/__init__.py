"""FP64 CPU oracle of the P3M step (test infrastructure only; see oracle.py)."""
from . import oracle  # noqa: F401
