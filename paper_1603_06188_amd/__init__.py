"""MI355X-native explicit APIC-MPM step (arXiv 1603.06188).

The compute path is the HIP library ``libapic.so`` (sources in ``csrc/``,
C ABI in ``include/apic.h``); ``binding`` marshals arguments to it and
``scenes`` draws seeded synthetic inputs.  The binding is imported on first
use so that ``scenes`` can be used without a GPU.
"""
import importlib

__all__ = ["binding", "scenes"]


def __getattr__(name):
    if name in ("binding", "scenes"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
