"""Storage of FP32 vector sets at the C ABI (test helper).

One FP32 vector is a plain [3][Vh] complex64 array.  A set of two or more
interleaves them in pairs: pair q holds right-hand sides 2q and 2q + 1 as a
[3][Vh] array of (rhs 2q, rhs 2q + 1) complex64 pairs, so element (r, c, eo)
is the complex64 at ((r // 2) * 3 * Vh + c * Vh + eo) * 2 + r % 2; an odd
count leaves the second half of the last pair unused.  FP64 sets are plain
[nrhs][3][Vh].  pack / unpack convert between that storage and [nrhs][3][Vh].
"""

import numpy as np


def pack(v):
    """[nrhs][3][Vh] complex64 -> the ABI storage ([npair][3][Vh][2] for nrhs >= 2)."""
    v = np.asarray(v, dtype=np.complex64)
    nrhs = v.shape[0]
    if nrhs < 2:
        return np.ascontiguousarray(v)
    out = np.zeros(((nrhs + 1) // 2, 3, v.shape[2], 2), dtype=np.complex64)
    out[:, :, :, 0] = v[0::2]
    out[: nrhs // 2, :, :, 1] = v[1::2]
    return out


def unpack(x, nrhs, Vh):
    """The ABI storage of nrhs FP32 vectors -> [nrhs][3][Vh]."""
    x = np.asarray(x)
    if nrhs < 2:
        return x.reshape(1, 3, Vh)
    p = x.reshape(-1, 3, Vh, 2)
    out = np.empty((nrhs, 3, Vh), dtype=x.dtype)
    out[0::2] = p[: (nrhs + 1) // 2, :, :, 0]
    out[1::2] = p[: nrhs // 2, :, :, 1]
    return out


def size(nrhs, Vh):
    """complex64 entries the ABI storage of nrhs FP32 vectors occupies."""
    return (nrhs if nrhs < 2 else (nrhs + 1) // 2 * 2) * 3 * Vh
