"""CPU oracle for CKKS hybrid key switching -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library in
``paper_2311_01598_amd``) never imports, links or executes anything here, and
this package never imports the product package.

Contents:
  * ``ks_oracle.c``  plain C (uint64 ``%`` arithmetic) key switching, NTT,
    basis conversion, key generation -- loaded through ctypes below;
  * ``bignum.py``    exact big-integer checks (CRT, decryption noise bound,
    basis-conversion and ModDown identities) using Python integers;
  * ``mlp.py``       float64 reference of the cost-model MLP.
"""
from .core import *  # noqa: F401,F403
