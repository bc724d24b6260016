"""MI355X (gfx950) implicit 2D3V particle-in-cell particle stage.

The computation lives in the HIP library ``libpic.so`` (C ABI in include/pic.h); this
package only builds it (``build.py``) and binds it (``binding.py``).
"""
from .binding import Context, PicError, init_grid, load_library  # noqa: F401
