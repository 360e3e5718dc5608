"""Seeded synthetic inputs shared by the library's tests, benchmark and the
oracle.  Holds no DMRG arithmetic: only sector-dimension recipes, random
numbers and the named workload presets.

Sector dimensions ("binomial rule"): at a bond with l spin-1/2 sites on its
left and N-l on its right, the sector of left charge q (q = 2 S^z of the
left block; charges are left-accumulated, see the library header) can hold
at most w_q = min(C(l, (l+q)/2), C(N-l, (N-l+q_t-q)/2)) states, q_t being the
target charge.  A bond of size m gets m_q = w_q when sum w_q <= m, otherwise
the largest-remainder apportionment of m in proportion to w_q, capped at
m_q <= w_q (ties in the remainder go to the smaller charge).

Physical basis of spin-1/2: index 0 = down (q = -1), index 1 = up (q = +1).
"""
from math import comb
import numpy as np

SPIN_HALF_Q = (-1, 1)
TRIVIAL_Q = (0, 0)   # no symmetry (used by the transverse-field Ising pins)


def _count(n, q):
    if n < 0 or (n + q) % 2 or abs(q) > n:
        return 0
    return comb(n, (n + q) // 2)


def binomial_bond(N, l, m, q_target=0):
    """Sector dims {q: m_q} of bond l (l sites on the left) for a chain of N
    spin-1/2 sites, truncated to m states by the binomial rule."""
    w = {}
    for q in range(-l, l + 1):
        c = min(_count(l, q), _count(N - l, q_target - q))
        if c > 0:
            w[q] = c
    total = sum(w.values())
    if total <= m:
        return dict(w)
    quota = {q: m * c / total for q, c in w.items()}
    out = {q: min(int(np.floor(quota[q])), w[q]) for q in w}
    left = m - sum(out.values())
    order = sorted(w, key=lambda q: (-(quota[q] - np.floor(quota[q])), q))
    while left > 0:
        progressed = False
        for q in order:
            if left == 0:
                break
            if out[q] < w[q]:
                out[q] += 1
                left -= 1
                progressed = True
        if not progressed:
            break
    return {q: n for q, n in out.items() if n > 0}


def binomial_bonds(N, m, q_target=0, trivial=False):
    """Sector dims of every bond 0..N of a chain, at most m states each."""
    if trivial:
        return [{0: min(m, 2 ** min(l, N - l))} for l in range(N + 1)]
    return [binomial_bond(N, l, m, q_target) for l in range(N + 1)]


def _charge_counts(n, phys_q):
    """Number of product states of n sites per total charge."""
    cnt = {0: 1}
    for _ in range(n):
        nxt = {}
        for q, c in cnt.items():
            for s in phys_q:
                nxt[q + s] = nxt.get(q + s, 0) + c
        cnt = nxt
    return cnt


def counted_bonds(N, m, phys_q, q_target=0):
    """Sector dims of every bond for any local charges: at a bond with l sites
    on the left the weight of charge q is min(#left states of charge q,
    #right states of charge q_target - q), apportioned to m by largest
    remainder (the binomial rule generalised)."""
    out = []
    for l in range(N + 1):
        left, right = _charge_counts(l, phys_q), _charge_counts(N - l, phys_q)
        w = {q: min(c, right.get(q_target - q, 0)) for q, c in left.items()}
        w = {q: c for q, c in sorted(w.items()) if c > 0}
        total = sum(w.values())
        if total <= m:
            out.append(dict(w))
            continue
        quota = {q: m * c / total for q, c in w.items()}
        o = {q: min(int(np.floor(quota[q])), w[q]) for q in w}
        left_over = m - sum(o.values())
        order = sorted(w, key=lambda q: (-(quota[q] - np.floor(quota[q])), q))
        while left_over > 0:
            progressed = False
            for q in order:
                if left_over == 0:
                    break
                if o[q] < w[q]:
                    o[q] += 1
                    left_over -= 1
                    progressed = True
            if not progressed:
                break
        out.append({q: n for q, n in o.items() if n > 0})
    return out


def random_site_blocks(bl, br, phys_q, rng):
    """Gaussian blocks {(q_left, s): array} of one MPS site tensor between
    bonds with sector dicts bl, br (allowed charge combinations only)."""
    out = {}
    for qa in sorted(bl):
        for s, qs in enumerate(phys_q):
            qb = qa + qs
            if qb in br:
                out[(qa, s)] = rng.standard_normal((bl[qa], br[qb]))
    return out


def random_mps(N, m, seed, phys_q=SPIN_HALF_Q, q_target=0):
    """Bond sector dicts and Gaussian site blocks of a random MPS."""
    rng = np.random.default_rng(seed)
    if tuple(phys_q) == (-1, 1) or all(q == 0 for q in phys_q):
        bonds = binomial_bonds(N, m, q_target, trivial=all(q == 0 for q in phys_q))
    else:
        bonds = counted_bonds(N, m, phys_q, q_target)
    sites = [random_site_blocks(bonds[i], bonds[i + 1], phys_q, rng) for i in range(N)]
    return bonds, sites


def isometric_scale(sites, bonds, phys_q, center):
    """Haar-random isometries in place of the Gaussian blocks, so that
    environments built from them stay O(1): a site left of `center` maps each
    right sector onto orthonormal columns (the Q factor of its Gaussian
    (a, s) x b stack), a site right of center + 1 has orthonormal rows per
    left sector.  Sampling only; returns new dicts."""
    out = []
    for i, s in enumerate(sites):
        new = dict(s)
        if i < center:
            for qb in sorted({qa + phys_q[k] for (qa, k) in s}):
                parts = [(qa, k) for (qa, k) in sorted(s) if qa + phys_q[k] == qb]
                G = np.vstack([s[p] for p in parts])
                if G.shape[0] >= G.shape[1]:
                    Q, _ = np.linalg.qr(G)
                    r0 = 0
                    for p in parts:
                        n = s[p].shape[0]
                        new[p] = Q[r0:r0 + n].copy()
                        r0 += n
        elif i > center + 1:
            for qa in sorted({qa for (qa, k) in s}):
                parts = [(q, k) for (q, k) in sorted(s, key=lambda t: t[1]) if q == qa]
                G = np.hstack([s[p] for p in parts])
                if G.shape[1] >= G.shape[0]:
                    Q, _ = np.linalg.qr(G.T)
                    c0 = 0
                    for p in parts:
                        n = s[p].shape[1]
                        new[p] = Q[c0:c0 + n].T.copy()
                        c0 += n
        out.append(new)
    return out


def random_two_site_blocks(bl, br, phys_q, rng):
    out = {}
    for qa in sorted(bl):
        for s1, q1 in enumerate(phys_q):
            for s2, q2 in enumerate(phys_q):
                qb = qa + q1 + q2
                if qb in br:
                    out[(qa, s1, s2)] = rng.standard_normal((bl[qa], br[qb]))
    return out


def random_env_blocks(bond, deltas, rng, hermitian_pairs=None):
    """Gaussian environment blocks {(q_bra, w): [m(q), m(q - delta_w)]}."""
    out = {}
    for q in sorted(bond):
        for w, dw in enumerate(deltas):
            if (q - dw) in bond:
                out[(q, w)] = rng.standard_normal((bond[q], bond[q - dw]))
    return out


# ---------------------------------------------------------------------------
# named workloads (lattice sizes, couplings, bond dimensions and seeds)
# ---------------------------------------------------------------------------

WORKLOADS = {
    "chain16": dict(kind="chain", N=16, J=1.0, m=64, init_m=16, sweeps=4, seed=1,
                    desc="spin-1/2 Heisenberg open chain N=16, m<=64, 4 sweeps, one region"),
    "cyl8x4_m1024": dict(kind="square", Lx=8, Ly=4, J=1.0, m=1024, seed=2, center=15,
                         desc="Heisenberg 8x4 cylinder (snake order), centre two-site "
                              "H_eff at sites 15,16 (0-based), m=1024"),
    "cyl24x8_4reg": dict(kind="square", Lx=24, Ly=8, J=1.0, seed=3, regions=4,
                         schedule=[200, 200, 650, 650, 1100, 1100, 1550, 1550, 2000, 2000],
                         n_warmup=2,
                         desc="Heisenberg 24x8 cylinder, 4 real-space regions, m 200->2000"),
    "tri12x6": dict(kind="triangular", Lx=12, Ly=6, J=1.0, seed=4, m=3000,
                    desc="triangular XXZ 12x6 cylinder, m=3000"),
    "jq2_16x8": dict(kind="jq2", Lx=16, Ly=8, J=1.0, seed=5, m=4000, regions=8,
                     desc="J-Q2 16x8 cylinder, m=4000, 8 regions"),
}


def delta_grid(seed=4, n=5, lo=0.8, hi=1.2):
    return sorted(np.random.default_rng(seed).uniform(lo, hi, n).tolist())


def q_grid(seed=5, n=5, lo=0.0, hi=2.0):
    return sorted(np.random.default_rng(seed).uniform(lo, hi, n).tolist())
