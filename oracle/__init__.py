"""CPU oracle for the DLIC hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct reference of what the GPU path computes:
causal neighbourhood gather, the small fully connected density network, the
discretised logistic-mixture head, frequency-table quantisation, the
interleaved rANS coder with its wavefront order, the bitstream container,
and the mixture NLL used for retraining.  Floating point is FP64 except
where an integer is decided from floating point (frequency quantisation):
there the oracle follows the format's FP32 rule, in the kernel's precision.

Only the tests, the smoke check (``__graft_entry__.smoke``) and the CPU
baseline leg of ``bench.py`` may import this package.  The product path
(``paper_2207_05152_amd``) never imports it, and this package imports
nothing from the product path; the two share only the seeded input
generators in ``synth``.

Parity status of each function is stated in its module header.  Citations
name sections, equations, figures and tables of the DLIC paper (Barzen,
Glazov, Geistert, Sikora, "Accelerated Deep Lossless Image Coding with
Unified Parallelized GPU Coding Architecture", arXiv 2207.05152).
"""
from .window import (NEIGHBOURS, SKEW, scale, causal_features, pixel_features,
                     step_of, n_steps)
from .network import mlp_forward, mixture_head, N_MIX, N_OUT, LOG_SCALE_MIN
from .mixture import (bin_edges, sigmoid, mixture_cdf, log_pmf, pmf_table,
                      ideal_bits, ideal_bits_image)
from .freq import (PROB_BITS, M_TOTAL, M_PRIME, table_exact, sigma_lut32,
                   sigma_hat32, table_coords32, beta32, scale32, table_levels32,
                   table_full32)
from .rans import (RANS_L, group_rows, group_strips, canonical_order, rans_encode,
                   rans_decode, RansDecoder)
from .container import (HEADER_SIZE, pack_header, parse_header, fingerprint,
                         assemble, split_streams, image_flags, image_strips)
from .codec import (OracleCoder, encode_image, decode_image, cf_for_image,
                    params32_for_image, weights_fingerprint)
from .nll import nll_bits, nll_and_grad_fd, adam_update, sample_features, PARAM_ORDER
from . import softmax, volume

__all__ = [n for n in dir() if not n.startswith("_")]
