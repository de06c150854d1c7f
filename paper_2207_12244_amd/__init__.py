"""MI355X (gfx950) keyframe depth update of DeepFusion (arxiv 2207.12244).

The product is the HIP library ``libkf.so`` behind the C ABI of
``include/kf.h``; ``paper_2207_12244_amd.kf`` is its Python binding.
"""

from .kf import (  # noqa: F401
    Keyframe,
    KfConfig,
    KfError,
    KfFrameStats,
    LIB_PATH,
    load_library,
)
