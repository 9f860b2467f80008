"""MI355X-native Exp-ParaDiag: the C-ABI HIP library and its binding."""
from .expdiag import *  # noqa: F401,F403
from .expdiag import Batch, Solver, load, LIB_PATH  # noqa: F401
