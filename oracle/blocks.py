"""U(1) block-sparse bonds and tensors (oracle; test infrastructure only).

Charges are integers q = 2 S^z.  Bond charges are *left-accumulated*: the
charge of a bond state is the total charge of the sites to its left, so
every MPS tensor conserves q_left + q_phys = q_right (bond 0 carries q = 0,
bond N carries the target charge).

Storage is a plain dict of dense numpy blocks:
  site tensor     key (q_left, s)        block [m_left(q), m_right(q + q_s)]
  two-site tensor key (q_left, s1, s2)   block [m_left(q), m_right(q + q_s1 + q_s2)]
  environment L   key (q_bra, w)         block [m(q_bra), m(q_bra - delta_w)]
  environment R   key (q_bra, w)         block [m(q_bra), m(q_bra - delta_w)]
(bra index first; L[a, w, a'] and R[b, w, b'] as in the usual DMRG
"projected operators" of Sec. II).  Blocks are kept only for allowed charge
combinations; a missing allowed block means zeros.
"""
import numpy as np


class Bond:
    """Sectors (charge, dimension) of one bond, ascending in charge."""
    __slots__ = ("qs", "dims", "_d")

    def __init__(self, sectors):
        items = sectors.items() if isinstance(sectors, dict) else sectors
        items = sorted((int(q), int(n)) for q, n in items if int(n) > 0)
        self.qs = tuple(q for q, _ in items)
        self.dims = tuple(n for _, n in items)
        self._d = dict(items)

    def dim(self, q):
        return self._d.get(q, 0)

    def has(self, q):
        return q in self._d

    def total(self):
        return sum(self.dims)

    def offset(self, q):
        """Position of the first state of sector q in the bond's state list."""
        o = 0
        for qq, n in zip(self.qs, self.dims):
            if qq == q:
                return o
            o += n
        raise KeyError(q)

    def __eq__(self, other):
        return isinstance(other, Bond) and self.qs == other.qs and self.dims == other.dims

    def __repr__(self):
        return "Bond(%s)" % dict(zip(self.qs, self.dims))


def site_keys(bl, br, phys_q):
    return [(qa, s) for qa in bl.qs for s in range(len(phys_q)) if br.has(qa + phys_q[s])]


def two_site_keys(bl, br, phys_q):
    d = len(phys_q)
    return [(qa, s1, s2) for qa in bl.qs for s1 in range(d) for s2 in range(d)
            if br.has(qa + phys_q[s1] + phys_q[s2])]


def env_keys(bond, deltas):
    return [(q, w) for q in bond.qs for w in range(len(deltas)) if bond.has(q - deltas[w])]


def site_shape(key, bl, br, phys_q):
    qa, s = key
    return (bl.dim(qa), br.dim(qa + phys_q[s]))


def two_site_shape(key, bl, br, phys_q):
    qa, s1, s2 = key
    return (bl.dim(qa), br.dim(qa + phys_q[s1] + phys_q[s2]))


def flatten(blocks, keys, shapes):
    """Concatenate the blocks (row-major) in the given key order."""
    parts = []
    for k, sh in zip(keys, shapes):
        b = blocks.get(k)
        parts.append(np.zeros(sh).ravel() if b is None else np.asarray(b, float).ravel())
    return np.concatenate(parts) if parts else np.zeros(0)


def unflatten(vec, keys, shapes):
    out, o = {}, 0
    for k, sh in zip(keys, shapes):
        n = sh[0] * sh[1]
        out[k] = vec[o:o + n].reshape(sh).copy()
        o += n
    assert o == len(vec)
    return out


def norm(blocks):
    return float(np.sqrt(sum(float(np.sum(b * b)) for b in blocks.values())))
