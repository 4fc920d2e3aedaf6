"""MI355X-native tactile force field (TacSL, Section III-C) behind a C-ABI.

The compute path lives in ``libtacsl.so`` (hand-written HIP for gfx950); this
package is the thin Python binding over it.  Importing the package does not
load the library; the first call that needs it does, and raises if it is
missing.
"""
__all__ = ["workloads"]
