"""Helpers shared by the tests: conversions between Python integers (the
oracle's representation) and the int64 tensors of the GPU library.  No
generator arithmetic lives here."""
import numpy as np
import torch

MASK64 = (1 << 64) - 1


def ints_to_words(values, nwords=9):
    """list of non-negative ints -> int64 array [len, nwords] (little-endian words)."""
    a = np.zeros((len(values), nwords), dtype=np.uint64)
    for i, v in enumerate(values):
        for k in range(nwords):
            a[i, k] = (v >> (64 * k)) & MASK64
    return a.view(np.int64)


def words_to_ints(arr):
    a = np.ascontiguousarray(np.asarray(arr)).view(np.uint64)
    return [sum(int(a[i, k]) << (64 * k) for k in range(a.shape[1])) for i in range(a.shape[0])]


def records_to_tensor(recs, device="cuda"):
    """list of (x, pos, p) -> int64 [n, 10] device tensor."""
    a = np.zeros((len(recs), 10), dtype=np.uint64)
    for i, (x, pos, p) in enumerate(recs):
        for k in range(9):
            a[i, k] = (x >> (64 * k)) & MASK64
        a[i, 9] = pos | (p << 32)
    return torch.from_numpy(a.view(np.int64)).to(device)


def tensor_to_records(t):
    a = t.cpu().numpy().view(np.uint64)
    out = []
    for i in range(a.shape[0]):
        x = sum(int(a[i, k]) << (64 * k) for k in range(9))
        w = int(a[i, 9])
        out.append((x, w & 0xFFFFFFFF, w >> 32))
    return out


def u64_list(t):
    """int64 tensor holding uint64 bit patterns -> list of Python ints."""
    return [int(v) & MASK64 for v in t.cpu().numpy().reshape(-1).tolist()]
