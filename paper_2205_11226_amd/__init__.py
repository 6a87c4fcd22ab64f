"""Python binding of libskmmse.so: scalable K-MMSE error concealment on MI355X.

Argument marshalling only: every step of the concealment runs in the HIP
library.  Importing this package loads the library and fails loudly when it
has not been built (``python paper_2205_11226_amd/build.py``).
"""
from .api import (  # noqa: F401
    LIB_PATH, BLOCK_INFO_DTYPE, MODES, LAYER_BRL, LAYER_IDL, LAYER_HQL, LAYER_FILL,
    FLAG_CTX_RELAXED, FLAG_NO_HQL, FLAG_NO_CAND, FLAG_EMPTY_CTX, FLAG_HQL_SINGULAR, SkmError,
    Params,
    default_params, patch_params, Context, lib, exported_symbols, FrameDesc, OPT_GRAPHS, OPT_BATCH_STREAMS,
    OPT_GATE_GRID, OPT_HQL_GRID, OPT_BATCH_MODE, OPT_EST_VARIANT,
    OPT_GROUP_SPLIT,
)
