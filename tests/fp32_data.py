"""The oracle's hierarchy on the data the FP32 V-cycle stores (test helper)."""
import numpy as np


def _r32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def fp32_data(H):
    """The oracle hierarchy H with the data the FP32 cycle stores rounded to
    FP32: the shifts (kept in units of h) and every level's block inverses
    (factorised in FP64, then rounded).  The coarsest dense inverse stays
    FP64.  Rounding the stored data is what defines the FP32 form, so this
    changes inputs only.  H is modified in place and returned."""
    for l, L in enumerate(H.levels):
        if L.n_surr:
            L.shifts = _r32(L.shifts / L.h) * L.h
            L.assemble()
        H.inv[l] = _r32(H.inv[l])
    return H
