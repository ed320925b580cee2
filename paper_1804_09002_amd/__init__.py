"""MI355X-native CS decomposition (Zolo-csd) — Python binding of libzcsd.

The compute path lives in the HIP library ``libzcsd.so`` (C ABI declared in
``include/zcsd.h``); this package only marshals torch device tensors into it.
Import of the binding is lazy so that ``paper_1804_09002_amd.workloads`` (the
seeded input generators) can be used without a GPU.
"""

__all__ = ["csd", "csd_batched", "csd_backward", "CSDFunction", "lib", "workloads"]


def __getattr__(name):
    if name in ("csd", "csd_batched", "csd_backward", "CSDFunction", "lib", "zolo_pd",
                "zolo_coeffs", "Options", "Info", "ZcsdError"):
        from . import zcsd as _z
        return getattr(_z, name)
    raise AttributeError(name)
