"""MI355X-native EPIC/MOFF imaging hot path (grid -> 2D FFT -> polarisation
products -> accumulate) behind the C ABI of include/epic.h.

``paper_2301_09662_amd.epic`` is the ctypes binding of ``libepic.so``; it is
imported lazily so that building does not require the library to exist.
"""


def build(verbose: bool = False) -> str:
    from . import _build
    return _build.build(verbose=verbose)


def load():
    from . import epic
    return epic
