"""Host-side helpers for tests: dense contraction of trains copied back from the device.
(Test infrastructure; plain numpy.)"""
import numpy as np


def contract_tt(cores):
    """cores: list of [r_l, d, r_{l+1}] arrays -> dense vector, core 0 slowest index."""
    v = cores[0]
    for G in cores[1:]:
        v = np.tensordot(v, G, axes=([-1], [0]))
    return v.reshape(-1)


def contract_mpo(cores):
    """cores: list of [w_l, 4, w_{l+1}] arrays (physical index u*2 + j) -> dense matrix
    [output index, input index], core 0 carrying the most significant digit of both."""
    n = len(cores)
    v = cores[0].reshape(cores[0].shape[0], 2, 2, cores[0].shape[2])
    for G in cores[1:]:
        v = np.tensordot(v, G.reshape(G.shape[0], 2, 2, G.shape[2]), axes=([-1], [0]))
    v = v.reshape([2] * (2 * n))
    perm = list(range(0, 2 * n, 2)) + list(range(1, 2 * n, 2))
    return v.transpose(perm).reshape(2 ** n, 2 ** n)


def right_orthonormality_error(cores):
    """max over cores 1..n-1 of || G G^H - I || with G reshaped [r_l, d r_{l+1}]."""
    err = 0.0
    for G in cores[1:]:
        A = G.reshape(G.shape[0], -1)
        err = max(err, np.abs(A @ A.conj().T - np.eye(A.shape[0])).max())
    return err


def tt_eval(cores, idx_bits):
    """Value of a train at one multi-index given as per-core digits."""
    v = np.ones((1,), dtype=np.complex128)
    for G, b in zip(cores, idx_bits):
        v = v @ G[:, b, :]
    return v[0]
