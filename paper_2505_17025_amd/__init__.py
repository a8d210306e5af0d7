"""MI355X-native hot path of the locally adaptive non-hydrostatic shallow water
model (Firdaus & Behrens): HIP kernels behind a C ABI (include/swe_nh.h) with
a thin ctypes binding.

Importing the binding requires the built HIP library; the package itself
imports without it so that the build step can run first.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "libswe_nh.so")


def binding():
    """the ctypes binding module (raises ImportError if the library is not built)"""
    from . import swe_nh
    return swe_nh
