"""MI355X (gfx950) hot path of Anderson-accelerated seismic inversion.

The wave-equation calls (forward modelling, adjoint-state gradient, Born
and its adjoint) and the Anderson step run in hand-written HIP kernels
behind the C ABI of ``libaafwi.so`` (declared in ``include/aafwi.h``);
``_lib`` is the ctypes binding and ``inversion`` drives Algorithm 2 and
its comparators on top of it.  The binding is loaded on first use, so the
build module can be imported before the library exists.
"""
_EXPORTS = ("AA", "AafwiError", "Batch", "BatchAA", "CNN", "Context", "Reducer", "axpy", "blend", "scale", "K_ADJ_STEP", "K_BORN_STEP",
            "K_FWD_STEP", "K_REC_STEP", "LIB_PATH")


def __getattr__(name):
    if name in _EXPORTS:
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)


__all__ = list(_EXPORTS)
