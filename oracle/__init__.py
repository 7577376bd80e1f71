"""FP64 CPU oracle (test infrastructure only; see dcp.py)."""
from .dcp import *  # noqa: F401,F403
from .dcp import Params, Result, dehaze  # noqa: F401
