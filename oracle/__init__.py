"""CPU oracle for the homomorphic Softmax hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or run anything in
this package.  The product library (``paper_2410_11184_amd``) shares no code
with it: no kernels, headers, helpers, tables or constant generators.

Contents
  ring.c       plain C ring primitives (NTT, base conversion, Philox, samplers)
  params.py    prime rule and canonical root of unity
  encoding.py  canonical-embedding encode/decode (special FFT)
  ckks.py      RNS-CKKS keygen / encrypt / decrypt / homomorphic operations
  softmax.py   FP64 Softmax definition, precision metrics, plaintext twins of
               the paper's algorithms (main loop, SM, AUX, SM version B)
  polyfit.py   Chebyshev interpolation and weighted Remez approximations
"""
