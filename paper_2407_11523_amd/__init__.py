"""MI355X (gfx950) flooding-schedule GF(4) belief propagation decoders for surface codes.

Traditional LLR-BP4, Momentum-BP, AdaGrad-BP and EWAInit-BP (Chen, Yi, Liang, Wang,
"Improved Belief Propagation Decoding Algorithms for Surface Codes") over very large
batches of syndromes, as hand-written HIP kernels behind the C ABI of include/bp4.h.
"""
from ._lib import BP4Error, load
from .api import (Captured, Graph, MixedBatch, Params, UnrolledBP, UnrolledEWAInit, bookkeep, decode, decode_mixed,
                  decode_plain, prior_llr, sample, unrolled_forward, unrolled_loss, unrolled_sizes)

__all__ = ["BP4Error", "Captured", "Graph", "MixedBatch", "Params", "UnrolledBP", "UnrolledEWAInit", "bookkeep", "decode",
           "decode_mixed", "decode_plain", "load", "prior_llr", "sample", "unrolled_forward", "unrolled_loss",
           "unrolled_sizes"]
