"""MI355X-native hot path of arXiv 2503.03479: affine view simulation, ORB and
all-view-pair Hamming matching, as hand-written HIP kernels for gfx950 behind
the C ABI of include/xaffine.h (libxaffine.so in this directory)."""
from . import xaffine  # noqa: F401
from .xaffine import XAError, Plan, plan_image, sampling_grid  # noqa: F401
