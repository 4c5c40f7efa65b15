"""MI355X (gfx950) implementation of the FOSB hot path: dense EFIE assembly,
combination-technique two-sided solves and far-field variance, behind the C
ABI declared in include/fosb.h.  ``fosb`` is the Python binding."""

from . import fosb  # noqa: F401  (binding only; the library loads on first use)

__all__ = ["fosb"]
