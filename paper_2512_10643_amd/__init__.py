"""MI355X-native conversion of pure bosonic Gaussian states into matrix
product states (Gaussian SVD + projected-creation-operator mapping), with
amplitude and sampling sweeps.  The compute path is the HIP library
libgbs_mps.so behind the C ABI in include/gbs_mps.h."""
from ._lib import GbsError, LIB_PATH, EXPORTED_SYMBOLS  # noqa: F401

__all__ = ["GbsError", "LIB_PATH", "EXPORTED_SYMBOLS", "build", "GaussianMPS"]


def __getattr__(name):
    if name in ("build", "GaussianMPS"):
        from . import mps
        return getattr(mps, name)
    raise AttributeError(name)
