"""MI355X (gfx950) ViPer NL-COMM vector-perturbation precoding.

The hot path (preprocess -> most-promising paths -> path search + argmin ->
precode) and the exact sphere encoder run in hand-written HIP kernels behind
the C ABI of include/vp.h; the learned path proposal (module `learn`) sits
behind include/vp_learn.h.  This package only marshals torch device tensors."""
from .vp import (VP_DEMAP_REGION, VP_INCLUDE_ZERO, VP_PATHS_PER_VECTOR, VP_SE_EXACT, VP_SE_EXHAUSTED, VP_SE_NONE,  # noqa: F401
                 FxInputs, FxOut, Prep, SearchOut, SEOut, apply_user_tau, fx_quantize, fx_search, packed_size, paths_mop, precode, preprocess, search, sphere_encode,
                 tau_array, version)
