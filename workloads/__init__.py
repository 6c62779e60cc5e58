"""Seeded synthetic inputs (contours, poses, incident fields) shared by the
FP64 reference implementation and the GPU library.  No method arithmetic."""
from . import geometry, configs  # noqa: F401
