"""Byzantine-robust selection and the encrypted mask (the KGC's side of
Algorithm 1, "Masked-based Encrypted Sorting", Algorithm 2).

The KGC decrypts the pairwise distances, ranks the clients, and answers the
server with one mask ciphertext per client, Enc_pk(w_i) with w_i the
client's aggregation weight as a constant plaintext (1 for the client that
Krum or the distance-Median picks, 1/l for each of Multi-Krum's l picks, 0
otherwise).  The server multiplies every client's packed ciphertexts by its
mask and sums (lc_mask_aggregate), so it never learns which clients were
chosen.  Selection runs on the host in FP64: it is a sort of n numbers.

Readings where the paper is loose:
  * the Krum score of client i sums its n - c - 2 smallest distances to the
    others (Appendix, Krum); clients are ranked by it for all three rules;
  * Median takes rank ceil(n / 2) of that ranking (Algorithm 2's index read
    as 1-based), Multi-Krum takes ranks 1, 2, ... while fewer than l are
    taken and n - |chosen| > 2c + 2;
  * ties go to the lower client index (stable sort);
  * Multi-Krum's weights are 1/l, the average of the chosen updates.
"""
from __future__ import annotations

import numpy as np

RULES = ("krum", "multikrum", "median")


def distance_matrix(pair_values, n):
    """Symmetric n x n matrix from the P = n(n-1)/2 values in row-major
    upper-triangle order (pairs (0,1), (0,2), ..., (n-2,n-1))."""
    iu = np.triu_indices(n, k=1)
    D = np.zeros((n, n))
    D[iu] = pair_values
    return D + D.T


def krum_scores(D, c):
    n = D.shape[0]
    m = max(n - c - 2, 0)
    off = D[~np.eye(n, dtype=bool)].reshape(n, n - 1)  # row i without its diagonal
    return np.sort(off, axis=1, kind="stable")[:, :m].sum(axis=1)


def select(rule, D, c, l=None):
    """Chosen client indices in rank order."""
    if rule not in RULES:
        raise ValueError("rule must be one of %s" % (RULES,))
    n = D.shape[0]
    rank = np.argsort(krum_scores(D, c), kind="stable")
    if rule == "krum":
        return [int(rank[0])]
    if rule == "median":
        return [int(rank[-(-n // 2) - 1])]
    l = n if l is None else l
    take = 0
    while take < l and n - take > 2 * c + 2:
        take += 1
    return [int(i) for i in rank[:take]]


def weights(rule, chosen, n):
    w = np.zeros(n)
    w[chosen] = 1.0 / len(chosen) if rule == "multikrum" else 1.0
    return w


def mask_plaintexts(w, N, scale):
    """Constant plaintexts round(scale * w_i) (coefficient 0 of an N-coefficient
    polynomial; a constant polynomial holds that value in every slot)."""
    m = np.zeros((len(w), N), dtype=np.int64)
    m[:, 0] = np.round(np.asarray(w) * scale).astype(np.int64)
    return m
