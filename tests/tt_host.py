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


def random_train(rng, ranks, d=2):
    """Random complex train with the given bond dimensions [1, r_1, ..., r_{n-1}, 1]."""
    return [(rng.standard_normal((ranks[l], d, ranks[l + 1])) +
             1j * rng.standard_normal((ranks[l], d, ranks[l + 1]))) / np.sqrt(2 * d * ranks[l + 1])
            for l in range(len(ranks) - 1)]


def right_orthonormalize(cores):
    """The same tensor with cores 1..n-1 right-orthonormal (G G^H = I for G reshaped
    [r_l, d r_{l+1}]), by QR factorisations from the right; bond dimensions unchanged
    when every unfolding has full rank."""
    cores = [c.astype(np.complex128).copy() for c in cores]
    for l in range(len(cores) - 1, 0, -1):
        r0, d, r1 = cores[l].shape
        Q, R = np.linalg.qr(cores[l].reshape(r0, d * r1).conj().T)   # G = R^H Q^H
        k = Q.shape[1]
        cores[l] = Q.conj().T.reshape(k, d, r1)
        cores[l - 1] = np.tensordot(cores[l - 1], R.conj().T, axes=([-1], [0]))
    return cores


def upload_train(tb, b, cores, flags=0):
    """Writes host cores [r_l, d, r_{l+1}] into train b of a device TTBatch (capacity
    layout) together with its bond dimensions, and sets the batch's canonical-form flags."""
    import torch
    off = tb.core_off[b].cpu().numpy()
    ranks = tb.ranks[b].cpu().numpy().copy()
    ranks[0] = 1
    for l, G in enumerate(cores):
        ranks[l + 1] = G.shape[2]
        flat = torch.from_numpy(np.ascontiguousarray(G).reshape(-1)).to(tb.cores.dtype)
        tb.cores[int(off[l]):int(off[l]) + flat.numel()] = flat.to(tb.cores.device)
    tb.ranks[b] = torch.from_numpy(ranks).to(tb.ranks.device)
    tb.struct.flags = flags
    tb.struct.rank_max = max(tb.struct.rank_max, int(ranks[: len(cores) + 1].max()))


def bitrev_perm(n):
    """perm[u] = the index u with its n bits reversed."""
    u = np.arange(2 ** n)
    r = np.zeros_like(u)
    for t in range(n):
        r |= ((u >> t) & 1) << (n - 1 - t)
    return r
