"""Seeded synthetic inputs shared by the library's tests, the benchmark and
the oracle: meshes, face pairs and analytic initial fields.  Holds no flux
reconstruction arithmetic."""
from . import configs, fields, meshes  # noqa: F401
