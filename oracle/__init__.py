"""CPU oracle for CKKS hybrid key switching -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library in
``paper_2311_01598_amd``) never imports, links or executes anything here, and
this package never imports the product package.

Contents:
  * ``ks_oracle.c``   plain C (uint64 ``%`` arithmetic) key switching, NTT,
    basis conversion, key generation for 30-bit towers in 32-bit words;
  * ``ks_oracle64.c`` the same for ~60-bit towers in 64-bit words (exact
    unsigned __int128 products reduced with ``%``), with compressed keys;
  * ``core.py``       ctypes wrappers of the 32-bit oracle and exact
    big-integer checks (CRT, decryption noise bound) using Python integers;
  * ``core64.py``     ctypes wrappers of the 64-bit oracle;
  * ``mlp.py``        float64 reference of the cost-model MLP.
"""
from .core import *  # noqa: F401,F403
