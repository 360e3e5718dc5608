"""Inverse canonical MPS gauge and local measurements (Sec. IV; oracle, test
infrastructure only).

The gauge: every site tensor psi_j is an orthogonality centre (all of its
indices label orthonormal states) and every bond b carries the diagonal
V_b = Lambda_b^{-1} of inverse Schmidt values, so that

    |Psi> = psi_0 V_1 psi_1 V_2 ... V_{N-1} psi_{N-1},
    psi_j = Lambda_j Gamma_j Lambda_{j+1}   (Gamma-Lambda canonical form).

It is reached as the paper describes: from a state whose only centre is the
first site, combine the first two site tensors, decompose with two copies of
Lambda and one V = Lambda^{-1} in between (the split of Eqs. eqn:inverse,
eqn:isvd), multiply one Lambda into each neighbour, and repeat at every bond.

Measurements: an operator acting on sites i..k needs only those site
tensors, because everything outside is an orthonormal basis on either side:
  * single site: <O_j> = sum psi_j[a,s,b] O[s,t] psi_j[a,t,b];
  * sites i < k: the left transfer of Sec. II ("projected operators") from
    the identity on bond i through psi_i, then B_j = V_j psi_j for j = i+1..k
    (B_j is right-orthonormal), closed with the trace on bond k+1.
All tensors are real.
"""
import numpy as np

from .blocks import Bond
from .dmrg import (State, canonicalize_right, contract_two, svd_truncate, update_L)
from .mpo import op_charge


class InverseCanonical:
    """bonds[b] (b = 0..N), psi[j] (site tensors, dict keyed (q_left, s)),
    V[b] and lam[b] (dict q -> vector) for the inner bonds b = 1..N-1."""

    def __init__(self, bonds, psi, V, lam, phys_q, n_floored):
        self.bonds = bonds
        self.psi = psi
        self.V = V
        self.lam = lam
        self.phys_q = tuple(phys_q)
        self.N = len(psi)
        self.n_floored = n_floored


def plain_sites(st):
    """Site tensors of a State with V absorbed into the left neighbour of
    every bond that carries one (the same state, no V left)."""
    sites = [dict(s) for s in st.sites]
    for b, Vb in st.V.items():
        sites[b - 1] = {(qa, s): blk * Vb[qa + st.phys_q[s]][None, :] for (qa, s), blk in sites[b - 1].items()}
    return sites


def inverse_canonical(mpo, bonds, sites, q_target, cutoff=1e-14, eps=1e-4):
    """Convert the MPS (plain site tensors, any gauge) to the inverse
    canonical gauge.  Right-canonical form with the centre on site 0 first
    (normalised), then the split at bonds 1..N-1 in order, keeping every
    singular value >= cutoff * lambda_max (Lambda renormalised, V floored as
    in the split of the sweep)."""
    st = State(mpo, [Bond(b) if not isinstance(b, Bond) else b for b in bonds], [dict(s) for s in sites], q_target)
    canonicalize_right(st)
    pq = st.phys_q
    psi, V, lam, nfl = [None] * st.N, {}, {}, 0
    for i in range(st.N - 1):
        theta = contract_two(st.sites[i], st.sites[i + 1], pq)
        res = svd_truncate(theta, st.bonds[i], st.bonds[i + 2], pq, 1 << 30, "split", cutoff, eps)
        st.bonds[i + 1] = res.bond
        psi[i] = res.left
        st.sites[i + 1] = res.right
        V[i + 1] = res.V
        lam[i + 1] = res.lam
        nfl += res.n_floored
    psi[st.N - 1] = st.sites[st.N - 1]
    return InverseCanonical(list(st.bonds), psi, V, lam, pq, nfl)


def expect_site(ic, j, op):
    """<O> on site j: sum over blocks of psi_j[a, s, :] . psi_j[a, t, :] O[s, t]
    (only charge-conserving entries of O can contribute)."""
    pq = ic.phys_q
    d = len(pq)
    val = 0.0
    for (qa, s), Xs in ic.psi[j].items():
        for t in range(d):
            if op[s, t] != 0.0 and pq[s] == pq[t]:
                Xt = ic.psi[j].get((qa, t))
                if Xt is not None:
                    val += op[s, t] * float(np.sum(Xs * Xt))
    return val


def _operator_sites(terms, i, k, d, phys_q):
    """MPO tensors for sum_t c_t A_t(i) B_t(k) on sites i..k: one channel
    per term between i and k (charge of A_t), identity in between."""
    T = len(terms)
    Wi = np.zeros((1, d, d, T))
    Wk = np.zeros((T, d, d, 1))
    Wm = np.zeros((T, d, d, T))
    deltas = np.array([op_charge(A, phys_q) for (_, A, _) in terms], dtype=np.int64)
    for t, (c, A, B) in enumerate(terms):
        Wi[0, :, :, t] = A
        Wk[t, :, :, 0] = c * B
        Wm[t, :, :, t] = np.eye(d)
    return Wi, Wm, Wk, deltas


def correlator(ic, i, k, terms):
    """sum_t c_t <A_t(i) B_t(k)> for i < k; terms = [(c, A, B), ...] with d x d
    operators whose charges cancel pairwise."""
    assert 0 <= i < k < ic.N
    pq = ic.phys_q
    d = len(pq)
    Wi, Wm, Wk, deltas = _operator_sites(terms, i, k, d, pq)
    zero = np.zeros(1, dtype=np.int64)
    # identity on bond i: the states left of psi_i are orthonormal
    E = {(q, 0): np.eye(n) for q, n in zip(ic.bonds[i].qs, ic.bonds[i].dims)}
    E = update_L(E, ic.psi[i], Wi, pq, zero, deltas)
    for j in range(i + 1, k + 1):
        Vb = ic.V[j]
        E = {(q, w): Vb[q][:, None] * blk * Vb[q - deltas[w]][None, :] for (q, w), blk in E.items()}
        W = Wm if j < k else Wk
        E = update_L(E, ic.psi[j], W, pq, deltas, deltas if j < k else zero)
    # the states right of psi_k are orthonormal: close with the trace
    return float(sum(np.trace(blk) for (q, w), blk in E.items() if w == 0))


def heisenberg_exchange(ops):
    """S_i . S_k = Sz Sz + (Sp Sm + Sm Sp) / 2 as correlator terms."""
    return [(1.0, ops["Sz"], ops["Sz"]), (0.5, ops["Sp"], ops["Sm"]), (0.5, ops["Sm"], ops["Sp"])]


def oc_residuals(ic):
    """Largest deviations from the defining properties, per site j:
    sum_{a,s} psi[a,s,b] psi[a,s,b'] = lam_{j+1}[b]^2 delta_bb' (right index),
    sum_{s,b} psi[a,s,b] psi[a',s,b] = lam_j[a]^2 delta_aa' (left index),
    with lam = 1 on the outer bonds."""
    pq = ic.phys_q
    out = []
    for j in range(ic.N):
        bl, br = ic.bonds[j], ic.bonds[j + 1]
        lam_l = ic.lam.get(j, {q: np.ones(n) for q, n in zip(bl.qs, bl.dims)})
        lam_r = ic.lam.get(j + 1, {q: np.ones(n) for q, n in zip(br.qs, br.dims)})
        rr = {}
        ll = {}
        for (qa, s), X in ic.psi[j].items():
            qb = qa + pq[s]
            rr[qb] = rr.get(qb, 0.0) + X.T @ X
            ll[qa] = ll.get(qa, 0.0) + X @ X.T
        e = 0.0
        for qb, G in rr.items():
            e = max(e, float(np.max(np.abs(G - np.diag(lam_r[qb] ** 2)))))
        for qa, G in ll.items():
            e = max(e, float(np.max(np.abs(G - np.diag(lam_l[qa] ** 2)))))
        out.append(e)
    return out


def order_dx(ic, Lx, Ly, ops, snake):
    """Columnar dimer order of the J-Q2 study (Sec. III): the average over y of
    <S_r.S_{r+x}> - <S_{r-x}.S_r>/2 - <S_{r+x}.S_{r+2x}>/2 at r = (Lx/2 - 1, y)
    (zero-based: the centre bond of an even-length cylinder)."""
    xc = Lx // 2 - 1
    ex = heisenberg_exchange(ops)

    def bond(x, y):
        a, b = snake(x, y, Ly), snake(x + 1, y, Ly)
        return correlator(ic, min(a, b), max(a, b), ex)
    return sum(bond(xc, y) - 0.5 * bond(xc - 1, y) - 0.5 * bond(xc + 1, y) for y in range(Ly)) / Ly


def order_mz(ic, Lx, Ly, ops, snake, sublattice):
    """Sublattice magnetisation of the triangular study (Sec. III): <S^z>
    averaged over the sites (xc, y) of sublattice 0, xc = (Lx - 1)//2."""
    xc = (Lx - 1) // 2
    vals = [expect_site(ic, snake(xc, y, Ly), ops["Sz"]) for y in range(Ly) if sublattice(xc, y) == 0]
    return sum(vals) / len(vals)
