"""MI355X-native Laplace-transform shifted-system solver (flexible shifted
Krylov with a multigrid preconditioner).  The compute path is the HIP
library built from ``csrc/``; ``binding`` exposes its C ABI to Python."""
import importlib

__all__ = ["binding"]


def __getattr__(name):
    if name == "binding":
        return importlib.import_module(".binding", __name__)
    raise AttributeError(name)
