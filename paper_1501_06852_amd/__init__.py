"""MI355X (gfx950) solver for the block-preconditioned FGMRES stage solve of the
Phase-Field Crystal equation (Praetorius & Voigt).

The compute path is the HIP library libpfc.so (C ABI in include/pfc.h);
`paper_1501_06852_amd.pfc` is its ctypes binding.  The binding is imported
lazily so that building does not require the library to exist.
"""


def __getattr__(name):
    if name == "pfc":
        import importlib
        return importlib.import_module(".pfc", __name__)
    raise AttributeError(name)
