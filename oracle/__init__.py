"""CPU oracle for the quasi-F-split height pipeline -- TEST INFRASTRUCTURE ONLY.

Two tiers, both written from the paper (arXiv 2502.12428), sharing no code
with the HIP library:

* ``oracle.literal`` -- Algorithms 1, 2, 3 and 5 on Python integers over Z.
* ``oracle.fast``    -- the same algorithms in plain C (``qfs_oracle.c``),
  with g~^p formed in Z/p^2 (a reading: Delta_1 mod p depends only on g~^p
  mod p^2); pinned against ``oracle.literal`` and against closed forms.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.
"""
