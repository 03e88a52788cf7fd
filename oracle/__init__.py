"""FP64 CPU oracle of DET-LSH.  Test infrastructure only: see detlsh_oracle."""
from .detlsh_oracle import *  # noqa: F401,F403
from . import detlsh_oracle  # noqa: F401
