"""MI355X-native batched Lottery BP (+OSD) decoder.

The decoding runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/lbp.h`` (``liblbp.so``); this package only marshals arguments.
"""
from ._lib import (  # noqa: F401
    LbpError, load, MSG_FP32, MSG_FP16, MSG_INT8, SCALE_PAPER, SCALE_CONST, FLIP_MSG, FLIP_LLR,
    OSD_NONE, OSD_0, OSD_CS, FLAG_CONVERGED, FLAG_OSD, FLAG_OSD_INCONSISTENT,
    CN_RANDOM, CN_WORST, VN_PROPOSED, VN_Q_FIRST, VN_UNRELIABLE, VN_RANDOM, lottery_rule, msg_fixed,
)
from .decoder import Code, Decoder, DecoderParams, Plan  # noqa: F401
from .server import Server  # noqa: F401

__version__ = "0.1.0"
