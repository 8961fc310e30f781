"""MI355X engine for the associative bond-swap potential (arXiv 1912.08569).

``librc.so`` (HIP, gfx950) implements the hot path behind a C ABI
(``include/rc.h``); ``api`` is its Python binding and ``engine.System`` the
buffer-owning convenience layer.  Importing this package loads the library
and fails loudly if it has not been built.
"""
from . import _lib

_lib.load()

from . import api  # noqa: E402
from .api import *  # noqa: E402,F401,F403
from .engine import RunResult, System  # noqa: E402,F401
from .batch import Batch, BatchResult  # noqa: E402,F401
from .rigid import RigidBodies  # noqa: E402,F401

__version__ = "0.1.0"
