"""Hellmann-Feynman gradients of the DMRG energy (oracle; test infrastructure only).

For a normalised MPS with its orthogonality centre on site i,
E = sum L_i[a,w,a'] psi[a,s,b] W_i[w,s,t,w'] psi[a',t,b'] R_{i+1}[b,w',b'],
so the gradient with respect to the MPO tensor at fixed state is
G_i[w,s,t,w'] = sum L_i[a,w,a'] psi[a,s,b] psi[a',t,b'] R_{i+1}[b,w',b'].
If every Hamiltonian term's coupling sits on exactly one site tensor (the
builder puts it on the term's last operator), then dE/dtheta =
sum_i <G_i, dW_i/dtheta> = <Psi| dH/dtheta |Psi>.

This is not part of the paper (its Sec. III scans large parameter spaces);
it is pinned against exact Hellmann-Feynman values from exact
diagonalisation, homogeneity identities and finite differences.
"""
import numpy as np

from .blocks import Bond
from .dmrg import update_L, svd_gesvd


def site_gradient(L, R, psi, phys_q, dl, dr):
    """G[w, s, t, w'] for the single-site centre psi[(q_a, s)] between L and R."""
    d = len(phys_q)
    G = np.zeros((len(dl), d, d, len(dr)))
    for (qa, w), Lb in L.items():
        qk = qa - dl[w]
        for s in range(d):
            Pb = psi.get((qa, s))
            if Pb is None:
                continue
            qb = qa + phys_q[s]
            for t in range(d):
                Pk = psi.get((qk, t))
                if Pk is None:
                    continue
                qbk = qk + phys_q[t]
                X = Pb.T @ Lb @ Pk           # [b, b']
                for w2 in range(len(dr)):
                    if qb - qbk != dr[w2]:
                        continue
                    Rb = R.get((qb, w2))
                    if Rb is None:
                        continue
                    G[w, s, t, w2] += float(np.sum(X * Rb))
    return G


def move_center_right(st, i):
    """Exact single-site gauge move of the centre from site i to i+1."""
    pq = st.phys_q
    d = len(pq)
    bl, br = st.bonds[i], st.bonds[i + 1]
    A, carry, dims = {}, {}, {}
    for qb in br.qs:
        rows = [(s, qb - pq[s]) for s in range(d) if bl.has(qb - pq[s]) and (qb - pq[s], s) in st.sites[i]]
        if not rows:
            continue
        M = np.vstack([st.sites[i][(qa, s)] for (s, qa) in rows])
        U, lam, Vt = svd_gesvd(M)
        r0 = 0
        for (s, qa) in rows:
            A[(qa, s)] = U[r0:r0 + bl.dim(qa)]
            r0 += bl.dim(qa)
        carry[qb] = lam[:, None] * Vt
        dims[qb] = len(lam)
    nxt = {}
    for (qb, s2), Y in st.sites[i + 1].items():
        if qb in carry:
            nxt[(qb, s2)] = carry[qb] @ Y
    st.sites[i], st.sites[i + 1] = A, nxt
    st.bonds[i + 1] = Bond(dims)
    st.L[i + 1] = update_L(st.L[i], A, st.mpo.W[i], pq, st.dl(i), st.dl(i + 1))


def mpo_gradients(st):
    """Measurement sweep: the state's centre must be on site 0 with valid right
    environments.  Returns [G_0, ..., G_{N-1}] and leaves the centre on the
    last site."""
    Gs = []
    for i in range(st.N):
        Gs.append(site_gradient(st.L[i], st.R[i + 1], st.sites[i], st.phys_q,
                                st.dl(i), st.dl(i + 1)))
        if i + 1 < st.N:
            move_center_right(st, i)
    return Gs


def coupling_gradient(Gs, dWs):
    """dE/dtheta = sum_i <G_i, dW_i/dtheta>."""
    return float(sum(np.sum(G * dW) for G, dW in zip(Gs, dWs)))
