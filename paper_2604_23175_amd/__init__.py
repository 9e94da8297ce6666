"""MI355X-native multi-area WLS state estimation (arXiv 2604.23175 hot path).

The compute path is the HIP library libmase.so (include/mase.h); `mase` is
its Python binding.  `warmstart` holds the learned warm-start extension.
"""
from . import mase  # noqa: F401
from .mase import Mase, MaseError, load  # noqa: F401
