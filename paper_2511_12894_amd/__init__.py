"""MI355X-native ratio-filter reconstruction of matched-filter SNR series
(Murakami, Ghosh, Morisaki, arXiv 2511.12894).

The compute path is librf.so (hand-written HIP for gfx950) behind the C ABI in
include/rf.h; `rf` is its ctypes binding and `synth` makes seeded inputs.
"""
__all__ = ["rf", "synth"]
