"""MI355X-native SVGD / sSVGD full-waveform-inversion hot path.

The compute path lives in ``libvip.so`` (hand-written HIP for gfx950, C-ABI
declared in ``include/vip.h``).  ``binding`` wraps that ABI with ctypes and
torch device tensors; importing this package does not load the library, so the
seeded input generators (``synth``) and workload definitions (``configs``)
work on machines without a GPU.  Every compute call fails loudly when the
library is missing.
"""
__all__ = ["configs", "synth"]
