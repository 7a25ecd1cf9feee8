"""swgn: per-frame Gauss-Newton warp-field solve on MI355X (gfx950).

The compute path is the HIP library libswgn.so (C ABI in include/swgn.h);
this package only builds it (`build`) and binds it (`swgn`).
"""
from . import swgn  # noqa: F401
from .swgn import Stream, SwConfig, SwError, config_for, sw_config_default  # noqa: F401
