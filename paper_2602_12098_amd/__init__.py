"""MI355X (gfx950) ViPer NL-COMM vector-perturbation precoding.

The hot path (preprocess -> most-promising paths -> path search + argmin ->
precode) runs in hand-written HIP kernels behind the C ABI of include/vp.h;
this package only marshals torch device tensors to it."""
from .vp import (VP_INCLUDE_ZERO, Prep, SearchOut, packed_size, paths_mop, precode, preprocess,  # noqa: F401
                 search, version)
