"""FP64 CPU oracle (test infrastructure only; see ``oracle.tucker``)."""
from .tucker import *  # noqa: F401,F403
from .tucker import __all__  # noqa: F401
from . import learn  # noqa: F401,E402  (learned warm start, also test infrastructure)
