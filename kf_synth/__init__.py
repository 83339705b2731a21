"""Seeded synthetic inputs (RGB-D scans and volume shapes) shared by the tests and the
benchmark.  Holds no integration arithmetic."""
from .scenes import Frames, VolumeSpec  # noqa: F401
