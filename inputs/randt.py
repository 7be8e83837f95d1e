"""Seeded random tensors for unit-level parity tests."""

from __future__ import annotations

import numpy as np


def random_complex(shape, seed, scale=1.0):
    """Complex128 array with i.i.d. N(0, scale^2/2) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (scale / np.sqrt(2.0)) * (re + 1j * im)


def random_mpo_like(wl, d, wr, seed, density=0.3):
    """A sparse-ish complex (wl, d, d, wr) tensor with whole zero (wl, wr) blocks.

    MPO site tensors are block sparse over the channel pair (wl, wr); this
    imitates that so kernels that skip zero blocks are exercised.
    """
    rng = np.random.default_rng(seed)
    W = random_complex((wl, d, d, wr), seed + 7919)
    keep = rng.random((wl, wr)) < density
    keep[0, 0] = True
    keep[-1, -1] = True
    return W * keep[:, None, None, :]


def random_hermitian_env(m, w, seed):
    """(m, w, m) environment whose every w-slice is Hermitian."""
    A = random_complex((m, w, m), seed)
    return 0.5 * (A + np.conj(np.transpose(A, (2, 1, 0))))
