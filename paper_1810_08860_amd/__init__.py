"""MI355X-native disk-blended light field renderer (Overbeck et al. 2018, Sec. 4).

The product is the HIP library ``liblf.so`` behind the C ABI in
``include/lf.h``; :mod:`paper_1810_08860_amd.lf` is its thin ctypes binding.
"""
from . import lf  # noqa: F401
from .lf import (LFError, lf_debug_candidates, lf_last_error, lf_load_views, lf_query,  # noqa: F401
                 lf_render, lf_render_reference, lf_set_tune, lf_stereo_eyes)
