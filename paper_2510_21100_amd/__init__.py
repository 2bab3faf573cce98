"""HistRetinex (arXiv 2510.21100) histogram pipeline on MI355X (gfx950).

The work runs in libhistretinex.so (hand-written HIP, C ABI in
include/histretinex.h); this package marshals torch tensors into it.
"""

from .api import (  # noqa: F401
    Params,
    Workspace,
    workspace,
    build_hist,
    build_hist_batch,
    solve,
    match,
    equalize,
    enhance,
    enhance_batch,
    enhance_batch_noalloc,
)
