"""FP64 / exact-integer CPU oracle of the Nacrith per-token probability pipeline.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the HIP path is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may import it; the
product path (the HIP library and its Python binding) never imports, links or calls anything here,
and this package imports nothing from the product.  The two share only the seeded input generator
in ``synth``, which holds none of the method's arithmetic.

Modules, each citing the passage of arXiv 2602.19626 it follows:

- ``transformer``  section 3.2 Eq. (lm) and section 3.10: FP64 decoder with the sliding KV cache.
- ``ngram``        section 3.5: interpolated token n-gram, orders 1..K, 64-slot continuation cap.
- ``head``         section 3.7 bias head, section 3.6 mixer, section 3.8 skip statistics, and the
                   softmax-gated ensemble gradients of the differentiation workload.
- ``cdf``          section 3.4: CDF-24 quantisation in exact integer arithmetic.
- ``coder``        section 3.9: 32-bit Witten-Neal-Cleary arithmetic coder on Python integers.
- ``pipeline``     Algorithm 1 and its decompression mirror (section 3.1).

Parity status of each function is stated in its module header; conventions that only the oracle
and the GPU path agree on (eviction tie-break, warmup/skip placement, BOS) are "parity unpinned".
"""
