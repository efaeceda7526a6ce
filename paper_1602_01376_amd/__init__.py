"""MI355X (gfx950) INV-ASKIT factor/solve of lambda*I + K~.

Submodules:
  setup    seeded CPU problem generator (points, ball tree, skeletons, P)
  binding  ctypes binding of the HIP C-ABI library libinvaskit.so
The binding is imported on first use so the setup works without a GPU.
"""
__all__ = ["setup", "binding"]


def __getattr__(name):
    if name in ("binding", "setup"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
