"""Helpers shared by the GPU tests (device transfers and error bounds)."""
import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def dev(x):
    import paper_2203_10879_amd as sr

    return sr.colmajor(np.asfortranarray(x))


def host(t):
    import paper_2203_10879_amd as sr

    return sr.to_numpy(t)


def empty(m, n, c64=False):
    import torch

    import paper_2203_10879_amd as sr

    return sr.colmajor_empty(m, n, torch.complex64 if c64 else torch.complex128)


def gemm_bound(a_abs, b_abs, k, u):
    """First-order componentwise bound for a complex dot product of length k."""
    return (k + 4) * u * np.sqrt(2.0) * (a_abs @ b_abs)


def rand_c(rng, shape):
    return np.asfortranarray(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def phase_align(q, qref):
    """q * diag(d) with d the unimodular phases that best match qref column-wise."""
    d = np.sum(q.conj() * qref, axis=0)
    d = d / np.abs(d)
    return q * d[None, :]
