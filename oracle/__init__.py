"""CPU oracle for the cache-friendly truncated FFT hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
in this directory.  The product (the HIP library and its Python binding) never
does, and this directory imports nothing from the product.

Contents
  tft_oracle  plain Python definitions over exact integers (small and medium
              sizes): eq. (1) of Sect. 2, the TFT/ITFT definitions of Sect. 2,
              the polynomial product of Sect. 2, schoolbook products in Z[x]
              and (Z/mZ)[x].
  coracle     the same definitions in plain C (``coracle.c``), for sampled
              outputs at the benchmark sizes.

Every function states the passage it follows.  Where a function has no pin
other than itself it says "parity unpinned"; at present every function is
pinned by the tests in ``tests/test_oracle_pins.py``.
"""
