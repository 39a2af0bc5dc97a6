"""Plain CPU mirror of the Lanczos-based low-rank correction method
(TEST INFRASTRUCTURE ONLY).

Written from Sec. II of the paper, in its order and notation, with exact
sparse solves.  It exists to pin the oracle against the method: at full
interface rank the method must reproduce diag(H^{-1}) exactly (eqs. (8)-(9)).

Steps, for one domain with interface (separator) set C and subdomain set B:
  eq. (4)   split H into B (block diagonal over subdomains), E and C;
  eq. (13)  diag(B^{-1}) once, by inverting each small subdomain block;
  eqs. (10)-(12)  the "matrix-vector" product with X = H^{-1} - blkdiag(B^{-1},0):
            solve H v = q, w = blkdiag(B^{-1},0) q, u = v - w;
  Sec. II.A bilinear (complex-symmetric) Lanczos: (q,u) = q^T u without
            conjugation, principal square root for the "norm", every product
            bilinear including the full re-orthogonalization (two classical
            Gram-Schmidt passes);
  after eq. (13)  diag(Q T Q^T) accumulated from three Lanczos vectors at a
            time: alpha_j q_j*q_j + 2 beta_{j+1} q_j*q_{j+1} summed over the
            accepted steps (q_0 = 0; no term with the residual beyond T);
  end of Sec. II.C  recursion: diag(B^{-1}) of a large subdomain comes from
            the same method applied to it, splitting alternately along x and y.

Readings of the text (each also listed with the design notes):
  * separators are one site wide and lie at p with (p+1) % s == 0, p < L-1,
    so subdomains are at most s sites along every axis (Fig. 1 layout);
  * the start vector is a seeded random complex vector (the paper is silent);
  * stop when the residual of the new Lanczos vector has fallen to tol times
    |u| in the 2-norm (the L2-norm criterion of Sec. II.C), or after m + extra
    steps ("5 or 10 extra iterations").
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .dyson import hamiltonian


def separator_positions(L: int, s: int):
    """One-site separator planes along an axis of length L for subdomain edge s."""
    return [p for p in range(L) if (p + 1) % s == 0 and p < L - 1]


def plan_boxes(dims, s, partition="nested"):
    """Domain tree.  Each node: dict(level, box=[(lo,hi) per axis], splits=
    [(axis, pos), ...]).  'single' puts every separator into the root (one
    level of domain decomposition, Fig. 1); 'nested' splits one plane at a
    time through the longest axis, nearest its middle, which alternates
    (d_x, d_y) = (2,1), (1,2), ... on square domains (end of Sec. II.C)."""
    dims = tuple(int(L) for L in dims)
    seps = [separator_positions(L, s) for L in dims]
    nodes = []

    def rec(box, level):
        cands = [[p for p in seps[a] if box[a][0] < p < box[a][1] - 1]
                 for a in range(len(dims))]
        if not any(cands):
            nodes.append(dict(level=level, box=box, splits=[]))
            return
        if partition == "single":
            splits = [(a, p) for a in range(len(dims)) for p in cands[a]]
        else:
            ext = [box[a][1] - box[a][0] if cands[a] else -1 for a in range(len(dims))]
            a = int(np.argmax(ext))                      # first longest axis
            mid = (box[a][0] + box[a][1] - 1) / 2.0
            p = min(cands[a], key=lambda q: (abs(q - mid), q))
            splits = [(a, p)]
        nodes.append(dict(level=level, box=box, splits=splits))
        # children: the sub-boxes between split planes
        edges = []
        for a in range(len(dims)):
            ps = sorted(p for (b, p) in splits if b == a)
            lo, hi = box[a]
            segs, cur = [], lo
            for p in ps:
                segs.append((cur, p))
                cur = p + 1
            segs.append((cur, hi))
            edges.append(segs)
        for seg in itertools_product(edges):
            rec(list(seg), level + 1)

    rec([(0, L) for L in dims], 0)
    return nodes


def itertools_product(edges):
    import itertools
    # slowest axis outermost so children come out in natural order
    for combo in itertools.product(*edges[::-1]):
        yield tuple(combo[::-1])


def _box_sites(dims, box):
    """Natural indices (x fastest) of the sites of a box, in box-natural order."""
    import itertools
    strides = np.cumprod((1,) + tuple(dims[:-1]))
    rng = [range(lo, hi) for (lo, hi) in box]
    out = []
    for c in itertools.product(*rng[::-1]):
        c = c[::-1]
        out.append(int(sum(ci * st for ci, st in zip(c, strides))))
    return np.array(out, dtype=np.int64)


def _interface_mask(dims, box, splits):
    """True for the box's sites lying on one of its split planes."""
    import itertools
    rng = [range(lo, hi) for (lo, hi) in box]
    mask = []
    for c in itertools.product(*rng[::-1]):
        c = c[::-1]
        mask.append(any(c[a] == p for (a, p) in splits))
    return np.array(mask, dtype=bool)


def bilinear_lanczos_diag(xmatvec, q1, kmax, tol):
    """Sec. II.A / II.C: bilinear Lanczos on X with full re-orthogonalization,
    returning diag(Q_k T_k Q_k^T), the steps taken and (alpha, beta)."""
    n = q1.shape[0]
    q = q1 / np.sqrt(q1 @ q1)               # principal square root of q^T q
    q_prev = np.zeros(n, dtype=np.complex128)
    beta = 0.0 + 0.0j
    Q = []
    D = np.zeros(n, dtype=np.complex128)
    alphas, betas = [], []
    steps = 0
    for j in range(kmax):
        Q.append(q)
        u = xmatvec(q)                       # eqs. (10)-(12)
        alpha = q @ u                        # (q, u)_C = q^T u, no conjugate
        r = u - alpha * q - beta * q_prev    # three-term recurrence
        Qm = np.array(Q)
        for _ in range(2):                   # full bilinear re-orthogonalization
            r = r - Qm.T @ (Qm @ r)
        # three-vector diagonal update: alpha_j q_j.q_j + 2 beta_j q_{j-1}.q_j
        D += alpha * q * q
        if j > 0:
            D += 2.0 * beta * q_prev * q
        alphas.append(alpha)
        steps = j + 1
        if np.linalg.norm(r) <= tol * np.linalg.norm(u):
            break
        beta = np.sqrt(r @ r)
        betas.append(beta)
        q_prev, q = q, r / beta
    return D, steps, np.array(alphas), np.array(betas)


def lowrank_diag(dims, d, t, s, partition="single", extra_steps=10, tol=1e-10,
                 seed=0, max_rank=None, return_info=False):
    """diag(H^{-1}) by the low-rank correction method with exact sparse solves.

    dims: lattice shape (x fastest), d: diagonal of H (one frequency),
    t: hopping, s: subdomain edge.  max_rank caps the Lanczos steps per domain
    (truncated rank; results are then approximate)."""
    dims = tuple(int(L) for L in dims)
    d = np.asarray(d, dtype=np.complex128)
    nodes = plan_boxes(dims, s, partition)
    G = np.zeros(d.shape[0], dtype=np.complex128)
    rng = np.random.default_rng(seed)
    info = []
    # bottom-up over the tree: deepest nodes first
    for node in sorted(nodes, key=lambda nd: -nd["level"]):
        idx = _box_sites(dims, node["box"])
        ldims = tuple(hi - lo for (lo, hi) in node["box"])
        Hn = hamiltonian(ldims, d[idx], t)
        if not node["splits"]:
            # a subdomain too small to split: diag(B^{-1}) by direct inversion
            G[idx] = np.diag(np.linalg.inv(Hn.toarray()))
            continue
        on_c = _interface_mask(dims, node["box"], node["splits"])
        ib = np.where(~on_c)[0]
        m = int(on_c.sum())
        lu_h = spla.splu(Hn)
        lu_b = spla.splu(Hn[ib][:, ib].tocsc())   # B: the subdomain blocks

        def xmatvec(q):
            v = lu_h.solve(q)                      # eq. (10)
            w = np.zeros_like(q)
            w[ib] = lu_b.solve(q[ib])              # eq. (11)
            return v - w                           # eq. (12)

        n = idx.shape[0]
        q1 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        kmax = m + extra_steps if max_rank is None else min(max_rank, m + extra_steps)
        D, steps, al, be = bilinear_lanczos_diag(xmatvec, q1, kmax, tol)
        # eq. (13): diag(H^{-1}) = diag(blkdiag(B^{-1}, 0)) + diag(Q T Q^T)
        base = G[idx].copy()                       # children filled diag(B^{-1})
        base[on_c] = 0.0
        G[idx] = base + D
        info.append(dict(level=node["level"], m=m, steps=steps, alpha=al, beta=be))
    return (G, info) if return_info else G


def interface_lanczos_diag(dims, d, t, s, partition="single", extra_steps=10, tol=1e-12,
                           seed=0, return_info=False):
    """diag(H^{-1}) from a Lanczos run on the Schur complement instead of on X
    (a variant derived from eqs. (5)-(7), not the paper's operator), exact
    sparse solves.  For a domain with interface C and subdomains B, eq. (6)
    reads H^{-1} = blkdiag(B^{-1}, 0) + [W; -I] S^{-1} [W^T, -I] with
    W = B^{-1} E, so diag(X) = diag(W S^{-1} W^T) inside the subdomains and
    diag(S^{-1}) on the interface.  Bilinear Lanczos on S (vectors of the
    interface size m, S p = C p - E^T B^{-1} E p: one subdomain solve per step),
    full re-orthogonalization (two classical Gram-Schmidt passes); with
    P^T P = I and S P = P H (H the projected Hessenberg matrix: the
    tridiagonal T plus the re-orthogonalization coefficients),
    S^{-1} = P H^{-1} P^T and diag(X) = diag(V H^{-1} V^T), V = [W P; P]:
    V's columns are the step's u = B^{-1} E p (subdomain sites) and p
    (interface).  H is inverted densely once per domain."""
    dims = tuple(int(L) for L in dims)
    d = np.asarray(d, dtype=np.complex128)
    nodes = plan_boxes(dims, s, partition)
    G = np.zeros(d.shape[0], dtype=np.complex128)
    rng = np.random.default_rng(seed)
    info = []
    for node in sorted(nodes, key=lambda nd: -nd["level"]):
        idx = _box_sites(dims, node["box"])
        ldims = tuple(hi - lo for (lo, hi) in node["box"])
        Hn = hamiltonian(ldims, d[idx], t)
        if not node["splits"]:
            G[idx] = np.diag(np.linalg.inv(Hn.toarray()))
            continue
        on_c = _interface_mask(dims, node["box"], node["splits"])
        ic, ib = np.where(on_c)[0], np.where(~on_c)[0]
        n, m = idx.shape[0], ic.shape[0]
        lu_b = spla.splu(Hn[ib][:, ib].tocsc())
        E = Hn[ib][:, ic]

        def smat(p):                                   # S p and u = B^{-1} E p
            u = lu_b.solve(E @ p)
            w = np.zeros(n, dtype=np.complex128)
            w[ic], w[ib] = p, -u
            return (Hn @ w)[ic], u

        q1 = rng.standard_normal(m) + 1j * rng.standard_normal(m)
        p = q1 / np.sqrt(q1 @ q1)                      # principal root of p^T p
        P, U = [], []
        kmax = m + max(extra_steps, (m + 7) // 8)
        Hh = np.zeros((kmax + 1, kmax), dtype=np.complex128)
        for j in range(kmax):
            P.append(p)
            sp, u = smat(p)
            U.append(u)
            Pm = np.array(P)
            h = Pm @ sp                                 # bilinear projections
            r = sp - Pm.T @ h
            h2 = Pm @ r
            r = r - Pm.T @ h2
            Hh[:j + 1, j] = h + h2
            if np.linalg.norm(r) <= tol * np.linalg.norm(sp):
                break
            beta = np.sqrt(r @ r)
            Hh[j + 1, j] = beta
            p = r / beta
        k = len(P)
        V = np.zeros((n, k), dtype=np.complex128)
        V[ic] = np.array(P).T
        V[ib] = np.array(U).T
        Dx = np.einsum("ij,jk,ik->i", V, np.linalg.inv(Hh[:k, :k]), V)
        base = G[idx].copy()
        base[on_c] = 0.0
        G[idx] = base + Dx
        info.append(dict(level=node["level"], m=m, steps=k))
    return (G, info) if return_info else G
