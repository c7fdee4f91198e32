"""Dense parity-check matrix written out element by element from a QC base
matrix (block (b, c) with shift s has a one at row b*Z + r, column
c*Z + (r + s) mod Z; Sec. 4.1 of the paper). An independent statement of H used
only to check the other implementations."""
import numpy as np


def dense_h(base, z):
    base = np.asarray(base)
    mb, nb = base.shape
    H = np.zeros((mb * z, nb * z), dtype=np.uint8)
    for b in range(mb):
        for c in range(nb):
            s = int(base[b, c])
            if s < 0:
                continue
            for r in range(z):
                H[b * z + r, c * z + (r + s) % z] = 1
    return H


def gf2_matvec(H, x):
    """H x over GF(2) for a batch x [F, n] -> [F, m]."""
    return (np.asarray(x, dtype=np.int64) @ H.T.astype(np.int64)) % 2
