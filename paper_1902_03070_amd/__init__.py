"""MI355X-native cosine-transform t-SVD / t-SVT / TNN-C completion.

The computation lives in the HIP library libtsvdmi.so (include/tsvdmi.h); this
package only marshals torch tensors to it.  Importing the functions below
requires the built library and raises ImportError otherwise.
"""
import importlib
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtsvdmi.so")


def __getattr__(name):
    if name.startswith("__") or name in ("_lib", "build", "serving"):
        raise AttributeError(name)
    mod = importlib.import_module(__name__ + "._lib")
    return getattr(mod, name)
