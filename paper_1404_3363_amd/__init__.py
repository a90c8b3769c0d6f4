"""ivr: the per-pixel hot path of isogeometric volume rendering on MI355X (gfx950).

The work runs in ``libivr.so`` (hand-written HIP kernels behind the C ABI of
include/ivr.h); this package only marshals arguments.
"""
from .ivr import (Renderer, IvrError, default_opts, load_library, EXPORTS, RenderOpts,
                  STAT_FIELDS)

__all__ = ["Renderer", "IvrError", "default_opts", "load_library", "EXPORTS", "RenderOpts",
           "STAT_FIELDS"]
