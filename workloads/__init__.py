"""Seeded synthetic input batches (no eigenvalue arithmetic); see
``workloads.generators``."""
from .generators import *  # noqa: F401,F403
from .generators import CHUNK, GENERAL_ENTRIES, SYMMETRIC_ENTRIES, SYMMETRIC_POS, SEEDS  # noqa: F401
