"""Philox4x32-10 counter-based bijection (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11), restated from its published
definition.

TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).  Integer-exact: numpy
uint64 holds every 32x32->64 product exactly.

Definition used here.  State: four 32-bit counter words (c0, c1, c2, c3) and two
32-bit key words (k0, k1).  One round multiplies c0 by 0xD2511F53 and c2 by
0xCD9E8D57 (full 64-bit products, split in hi/lo halves) and returns
    (hi(c2*M1) ^ c1 ^ k0,  lo(c2*M1),  hi(c0*M0) ^ c3 ^ k1,  lo(c0*M0)).
Between rounds the key is advanced by the Weyl constants (0x9E3779B9,
0xBB67AE85) modulo 2^32.  Ten rounds make one output block of four words.

Parity pin: bit-exact against rocRAND's independent host implementation of the
same engine (tests/test_oracle_noise.py).
"""

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(counter, key):
    """Apply the ten-round bijection.

    counter: integer array [..., 4] of 32-bit words (c0, c1, c2, c3).
    key:     pair (k0, k1) of 32-bit words.
    Returns a uint32 array [..., 4] with the four output words.
    """
    ctr = np.asarray(counter, dtype=np.uint64) & _LO
    c0, c1, c2, c3 = ctr[..., 0], ctr[..., 1], ctr[..., 2], ctr[..., 3]
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & _LO
            k1 = (k1 + _W1) & _LO
        p0 = c0 * _M0
        p1 = c2 * _M1
        c0, c1, c2, c3 = ((p1 >> _S32) ^ c1 ^ k0, p1 & _LO,
                          (p0 >> _S32) ^ c3 ^ k1, p0 & _LO)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)
