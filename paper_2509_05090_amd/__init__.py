"""MI355X-native QR-based CTMRG for C3v-symmetric honeycomb iPEPS
(arXiv 2509.05090).

The computation lives in libctm.so (HIP for gfx950, C interface in
include/ctm.h); ``paper_2509_05090_amd.ctm`` is its Python binding.
"""
__all__ = ["ctm"]
