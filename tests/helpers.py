"""Test-side glue: move block data between the oracle's dict-of-blocks form and
the library's flat layouts (using the library's own block tables), build
random bond problems from the shared seeded generators, and load the HIP
library."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1301_3494_amd import _lib as pl          # noqa: E402
from paper_1301_3494_amd import synth                # noqa: E402


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def blocks_to_flat(blocks, table, n, kind):
    """Scatter oracle blocks into a flat array using the library block table.
    ENV_R blocks are stored transposed (rows = ket)."""
    out = np.zeros(n)
    for key, off, rows, cols, ld in table:
        k = key[:2] if kind in (pl.SITE, pl.ENV_L, pl.ENV_R) else key
        b = blocks.get(k)
        if b is None:
            continue
        if kind == pl.ENV_R:
            b = b.T
        assert b.shape == (rows, cols), (key, b.shape, rows, cols)
        for r in range(rows):
            out[off + r * ld: off + r * ld + cols] = b[r]
    return out


def flat_to_blocks(vec, table, kind):
    out = {}
    for key, off, rows, cols, ld in table:
        k = key[:2] if kind in (pl.SITE, pl.ENV_L, pl.ENV_R) else key
        b = np.empty((rows, cols))
        for r in range(rows):
            b[r] = vec[off + r * ld: off + r * ld + cols]
        out[k] = b.T.copy() if kind == pl.ENV_R else b
    return out


def tables(bl, br, phys_q, dl=None, dr=None):
    """Library layout tables for a two-site problem on bonds (bl, br)."""
    B1, B2, P = pl.Bond(bl), pl.Bond(br), pl.Phys(phys_q)
    t = {}
    t["x"] = pl.layout(pl.TWO_SITE, B1, B2, P)
    if dl is not None:
        t["L"] = pl.layout(pl.ENV_L, B1, deltas=dl)
    if dr is not None:
        t["R"] = pl.layout(pl.ENV_R, B2, deltas=dr)
    return t, (B1, B2, P)


def mpo_site(mpo, i):
    return pl.MpoSite(mpo.W[i], mpo.deltas[i], mpo.deltas[i + 1])


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def say(*args):
    print(*args, flush=True)


def golden(key):
    """A stored exact reference value (tests/golden/exact_energies.json,
    written from the oracle by tests/golden/make_golden.py)."""
    import json
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_energies.json")) as f:
        return json.load(f)[key]


# ---------------------------------------------------------------- brute force on dense states
def dense_state(sites, bonds, N, V=None):
    """Brute-force contraction of an MPS into the 2^N amplitudes, index
    sum_i bit_i 2^i with bit_i = 1 for site i up (s = 1); V (optional) is
    applied on the bonds that carry one."""
    part = {0: np.ones((1, 1))}
    for j in range(N):
        new = {}
        rows = 1 << j
        for (qa, s), X in sites[j].items():
            if qa not in part:
                continue
            qb = qa + (-1, 1)[s]
            blk = part[qa] @ X
            tgt = new.setdefault(qb, np.zeros((2 * rows, X.shape[1])))
            tgt[s * rows:(s + 1) * rows] += blk
        if V is not None and (j + 1) in V:
            new = {q: blk * V[j + 1][q][None, :] for q, blk in new.items()}
        part = new
    (q, vec), = part.items()
    return vec[:, 0]


def dense_sz(psi, N, j):
    bits = (np.arange(psi.size) >> j) & 1
    return float(np.sum(psi ** 2 * np.where(bits == 1, 0.5, -0.5)))


def dense_exchange(psi, N, i, k):
    idx = np.arange(psi.size)
    bi, bk = (idx >> i) & 1, (idx >> k) & 1
    zz = np.sum(psi ** 2 * np.where(bi == bk, 0.25, -0.25))
    flip = idx ^ ((1 << i) | (1 << k))
    xy = 0.5 * np.sum(np.where(bi != bk, psi * psi[flip], 0.0))
    return float(zz + xy)
