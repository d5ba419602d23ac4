"""FP64 CPU oracle (test infrastructure only; see ``oracle.tucker``)."""
from .tucker import *  # noqa: F401,F403
from .tucker import __all__  # noqa: F401
