"""Order-independent digest of a set of packed states, evaluated with torch
(test bookkeeping, not part of the method).

The formula is the oracle's (``oracle.digest``): for a state of words
x_0 .. x_{w-1}, u = c_k + sum_i (x_i mod p) * a_k[i] (mod p) with
p = 2^31 - 1, and the digest is the pair of sums of u^3 + u (mod p) over the
set, k = 0, 1.  Every intermediate stays below 2^63, so int64 tensors hold it
exactly on any device.  ``table_digest`` walks a table's raw storage window by
window on the device, so a table far larger than host memory can be compared
with the oracle's digest of the reachable set."""
from __future__ import annotations

P = 0x7FFFFFFF
A = ((1103515245, 1664525013, 22695477, 134775813),
     (1013904223, 69069, 2147483629, 1566083941))
C = (12345, 987654321)


def digest_words(x, w: int) -> tuple[int, int]:
    """Digest of the rows of ``x`` (an int64 tensor of shape (n, >= w) holding
    word values in [0, 2^32)); n < 2^32."""
    import torch

    out = []
    for k in range(2):
        u = torch.full((x.shape[0],), C[k], dtype=torch.int64, device=x.device)
        for i in range(w):
            u = (u + (x[:, i] % P) * A[k][i] % P) % P
        f = ((u * u % P) * u + u) % P
        out.append(int(f.sum().item()) % P)
    return out[0], out[1]


def add(d, e) -> tuple[int, int]:
    return (d[0] + e[0]) % P, (d[1] + e[1]) % P


def table_digest(table, device, window_words: int = 1 << 28) -> tuple[int, tuple[int, int]]:
    """(number of occupied slots, digest of their keys) of a gx table, read
    through gx_table_copy_raw in windows of ``window_words`` words."""
    import torch

    info = table.info
    S, w = info.slot_words, info.words_per_state
    total = info.n_buckets * info.bucket_words
    window_words = max(S, window_words // S * S)
    buf = torch.empty(min(window_words, total), dtype=torch.int32, device=device)
    count, dig = 0, (0, 0)
    for first in range(0, total, window_words):
        n = min(window_words, total - first)
        part = buf[:n]
        table.copy_raw(part, first)
        slots = part.view(-1, S)
        occ = slots[slots[:, 0] != -1]  # -1 is the empty word 0xFFFFFFFF
        if occ.shape[0]:
            x = occ[:, :w].to(torch.int64) & 0xFFFFFFFF
            dig = add(dig, digest_words(x, w))
            count += occ.shape[0]
            del x
        del occ, slots
    torch.cuda.synchronize(device)
    return count, dig
