"""Oracle for G_ii(i w_k) = [H(i w_k)^{-1}]_ii  (TEST INFRASTRUCTURE ONLY).

The quantity is fixed by eq. (1) and the goal stated right after it (Sec. I):
H_ij = t on every nearest-neighbour bond, H_ii = i w_k + mu - V_i - Sigma_i(i w_k),
and only the diagonal of H^{-1} is wanted.  H is complex symmetric (real
off-diagonal, complex diagonal), never Hermitian, so no conjugation appears
anywhere below.  Everything is float64 / complex128.

Three independent evaluations of the diagonal (they share only the assembly):
  O1 diag_inv_dense   -- dense LAPACK inversion (the "original IDMFT code"
                         route of Sec. III), tiny lattices;
  O2 diag_inv_rgf     -- exact block-tridiagonal recursion over the slowest
                         axis (recursive Green's function), open lattices;
  O3 diag_inv_sampled -- sparse LU of H and unit-vector solves H x = e_i for a
                         chosen set of sites (eq. (14) restricted to samples).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# --------------------------------------------------------------------- eq. (1)
def assemble_diag(V, omega, sigma, mu):
    """Diagonal of H, eq. (1): d_i(k) = i w_k + mu - V_i - Sigma_i(i w_k).

    V [N] float, omega [K] float, sigma [K,N] complex -> d [K,N] complex128.
    """
    V = np.asarray(V, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.complex128)
    return (1j * omega[:, None] + mu) - V[None, :] - sigma


def assemble_diag_z(V, z, sigma, mu):
    """eq. (1) at complex energies z_k (Im z_k > 0) in place of i w_k, e.g. the
    real axis z_k = w_k + i eta (Sec. I notes the same matrix there):
    d_i(k) = z_k + mu - V_i - Sigma_i(z_k).  z [K] complex."""
    V = np.asarray(V, dtype=np.float64)
    z = np.asarray(z, dtype=np.complex128)
    sigma = np.asarray(sigma, dtype=np.complex128)
    return (z[:, None] + mu) - V[None, :] - sigma


def _bonds(dims, periodic=False):
    """Nearest-neighbour bonds (i, j), i < j in natural order (x fastest).

    Z = 2 D neighbours per interior site: 4 on the square lattice, 6 on the
    cubic one (Sec. I).  periodic: True wraps every axis, or one flag per axis
    (a wrapped axis adds the bond between sites L-1 and 0)."""
    dims = tuple(int(L) for L in dims)
    per = ([bool(periodic)] * len(dims) if np.ndim(periodic) == 0
           else [bool(x) for x in periodic])
    n = int(np.prod(dims))
    idx = np.arange(n).reshape(dims[::-1])          # [..., y, x]
    rows, cols = [], []
    for a in range(len(dims)):
        ax = len(dims) - 1 - a                      # numpy axis of lattice axis a
        L = dims[a]
        if L < 2:
            continue
        src = idx
        dst = np.roll(idx, -1, axis=ax)
        if not per[a]:
            sl = [slice(None)] * len(dims)
            sl[ax] = slice(0, L - 1)
            src, dst = src[tuple(sl)], dst[tuple(sl)]
        elif L == 2:
            # a ring of two sites has one bond, not two
            sl = [slice(None)] * len(dims)
            sl[ax] = slice(0, 1)
            src, dst = src[tuple(sl)], dst[tuple(sl)]
        rows.append(src.ravel())
        cols.append(dst.ravel())
    if not rows:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(rows), np.concatenate(cols)


def hamiltonian(dims, d, t, periodic=False):
    """Sparse H of eq. (1) for one frequency: t on bonds, d on the diagonal."""
    d = np.asarray(d, dtype=np.complex128)
    n = d.shape[0]
    r, c = _bonds(dims, periodic)
    off = sp.coo_matrix((np.full(r.shape[0], t, dtype=np.complex128), (r, c)),
                        shape=(n, n))
    return (off + off.T + sp.diags(d)).tocsc()


def dense_hamiltonian(dims, d, t, periodic=False):
    return hamiltonian(dims, d, t, periodic).toarray()


# -------------------------------------------------------------------- O1
def diag_inv_dense(dims, d, t, periodic=False, full=False):
    """O1: diag of the dense inverse (LAPACK), eq. (1) taken literally."""
    G = np.linalg.inv(dense_hamiltonian(dims, d, t, periodic))
    return G if full else np.diag(G).copy()


# -------------------------------------------------------------------- O2
def diag_inv_rgf(dims, d, t):
    """O2: exact diagonal of H^{-1} on an OPEN lattice by the block-tridiagonal
    recursive Green's function over the slowest axis.

    Ordering sites by slices of the slowest axis makes H block tridiagonal with
    diagonal blocks A_s (the slice's own lattice problem) and off-diagonal
    blocks t*I.  Left-connected blocks g_s = (A_s - t^2 g_{s-1})^{-1}, then the
    exact diagonal blocks run backwards: G_{nn} = g_n,
    G_{ss} = g_s + t^2 g_s G_{s+1,s+1} g_s.  Complex symmetric: transposes, not
    adjoints (all blocks here are symmetric)."""
    dims = tuple(int(L) for L in dims)
    d = np.asarray(d, dtype=np.complex128)
    n_slices = dims[-1]
    slice_dims = dims[:-1] if len(dims) > 1 else (1,)
    m = int(np.prod(slice_dims))
    D = d.reshape(n_slices, m)
    # in-slice hopping pattern
    r, c = _bonds(slice_dims) if len(dims) > 1 else (np.zeros(0, int), np.zeros(0, int))
    T = np.zeros((m, m), dtype=np.complex128)
    T[r, c] = t
    T[c, r] = t
    g = []
    prev = None
    for s in range(n_slices):
        A = T + np.diag(D[s])
        if prev is not None:
            A = A - (t * t) * prev
        prev = np.linalg.inv(A)
        g.append(prev)
    out = np.empty((n_slices, m), dtype=np.complex128)
    Gss = g[-1]
    out[-1] = np.diag(Gss)
    for s in range(n_slices - 2, -1, -1):
        Gss = g[s] + (t * t) * (g[s] @ Gss @ g[s])
        out[s] = np.diag(Gss)
    return out.reshape(-1)


# -------------------------------------------------------------------- O3
def nested_dissection_order(dims):
    """A fill-reducing permutation of the natural site order: split the box
    through the middle of its longest axis by a one-site plane, order the two
    halves first (recursively) and the plane last.  It only relabels the sites
    (H -> P H P^T), so the diagonal of the inverse is unchanged; it keeps the
    sparse LU of a 3-D lattice affordable."""
    dims = tuple(int(L) for L in dims)
    strides = np.cumprod((1,) + dims[:-1])
    out = []

    def block(lo, hi):
        grids = np.meshgrid(*[np.arange(a, b) for a, b in zip(lo, hi)], indexing="ij")
        return sum(g.ravel() * s for g, s in zip(grids, strides))

    def rec(lo, hi):
        ext = [b - a for a, b in zip(lo, hi)]
        ax = int(np.argmax(ext))
        if ext[ax] <= 3:
            out.append(block(lo, hi))
            return
        mid = (lo[ax] + hi[ax]) // 2
        h1 = list(hi)
        h1[ax] = mid
        l2 = list(lo)
        l2[ax] = mid + 1
        rec(list(lo), h1)
        rec(l2, list(hi))
        ls, hs = list(lo), list(hi)
        ls[ax], hs[ax] = mid, mid + 1
        out.append(block(ls, hs))

    rec([0] * len(dims), list(dims))
    return np.concatenate(out).astype(np.int64)


def diag_inv_sampled(dims, d, t, sites, periodic=False, order="natural"):
    """O3: G_ii for the given sites from one sparse LU of H and the unit solves
    H x^i = e^i of eq. (14), reading x^i_i.  order="nd" factors the
    nested-dissection relabelling P H P^T instead (no pivoting: every leading
    block of H has a positive definite imaginary part), the same numbers."""
    H = hamiltonian(dims, d, t, periodic)
    n = len(d)
    sites = np.asarray(sites, dtype=np.int64)
    if order == "nd":
        perm = nested_dissection_order(dims)
        where = np.empty_like(perm)
        where[perm] = np.arange(n)                 # position of site i in P H P^T
        lu = spla.splu(H[perm][:, perm].tocsc(), permc_spec="NATURAL", diag_pivot_thresh=0.0)
        rows = where[sites]
    else:
        lu = spla.splu(H)
        rows = sites
    out = np.empty(len(sites), dtype=np.complex128)
    for c0 in range(0, len(sites), 64):            # unit right-hand sides, 64 at a time
        r = rows[c0:c0 + 64]
        E = np.zeros((n, len(r)), dtype=np.complex128)
        E[r, np.arange(len(r))] = 1.0
        X = lu.solve(E)
        out[c0:c0 + len(r)] = X[r, np.arange(len(r))]
    return out


# -------------------------------------------------------------- closed forms
def closed_form_periodic(dims, z, t):
    """Uniform periodic lattice with constant diagonal z = i w + mu (V = Sigma = 0):
    plane waves diagonalise H, eigenvalue z + 2t sum_d cos(2 pi k_d / L_d), so
    G_ii = (1/N) sum_k 1 / (z + 2t sum_d cos(2 pi k_d/L_d)) for every i.
    (Closed form quoted for the uniform periodic lattice as a check.)"""
    grids = [2.0 * np.cos(2.0 * np.pi * np.arange(L) / L) if L > 2 else
             (np.array([1.0, -1.0]) if L == 2 else np.array([0.0])) for L in dims]
    eps = np.zeros(1)
    for g in grids:
        eps = (eps[:, None] + g[None, :]).ravel()
    return np.mean(1.0 / (z + t * eps))


def closed_form_uniform(dims, z, t, periodic):
    """Uniform lattice, constant diagonal z, each axis periodic or open: H is a
    sum over axes of commuting chain operators, so its eigenvectors are products
    of chain modes.  A periodic axis contributes plane waves (|psi_k(x)|^2 = 1/L,
    eigenvalue 2cos(2 pi k/L)), an open axis the sine modes of
    closed_form_open_uniform, and G_ii = sum over modes of the product of the
    squared mode values at site i over (z + t * sum of eigenvalues).
    Returns G_ii for all sites in natural order."""
    dims = tuple(int(L) for L in dims)
    wts, lams = [], []
    for L, p in zip(dims, periodic):
        x = np.arange(L)
        if p and L > 2:
            k = np.arange(L)
            wts.append(np.full((L, L), 1.0 / L))
            lams.append(2.0 * np.cos(2.0 * np.pi * k / L))
        else:
            n = np.arange(1, L + 1)
            wts.append((2.0 / (L + 1)) * np.sin(np.pi * np.outer(x + 1, n) / (L + 1)) ** 2)
            lams.append(2.0 * np.cos(np.pi * n / (L + 1)))
    out = np.zeros(tuple(dims), dtype=np.complex128)
    for modes in itertools.product(*[range(L) for L in dims]):
        lam = sum(lams[a][modes[a]] for a in range(len(dims)))
        w = wts[0][:, modes[0]]
        for a in range(1, len(dims)):
            w = np.multiply.outer(w, wts[a][:, modes[a]])
        out += w / (z + t * lam)
    return np.transpose(out).reshape(-1)


def closed_form_open_uniform(dims, z, t):
    """Uniform open lattice, constant diagonal z: the open-chain modes
    phi_n(x) = sqrt(2/(L+1)) sin(pi n (x+1)/(L+1)), eigenvalue 2 cos(pi n/(L+1)),
    give G_ii = sum_n prod_d phi_{n_d}(x_d)^2 / (z + t sum_d 2cos(pi n_d/(L_d+1))).
    Returns G_ii for all sites in natural order."""
    dims = tuple(int(L) for L in dims)
    phis, lams = [], []
    for L in dims:
        n = np.arange(1, L + 1)
        x = np.arange(L)
        phis.append(np.sqrt(2.0 / (L + 1)) * np.sin(np.pi * np.outer(x + 1, n) / (L + 1)))
        lams.append(2.0 * np.cos(np.pi * n / (L + 1)))
    out = np.zeros(tuple(dims), dtype=np.complex128)
    for modes in itertools.product(*[range(L) for L in dims]):
        lam = sum(lams[a][modes[a]] for a in range(len(dims)))
        w = np.ones(1)
        for a in range(len(dims)):
            w = np.multiply.outer(w, phis[a][:, modes[a]] ** 2) if a else phis[a][:, modes[a]] ** 2
        out += w / (z + t * lam)
    # out is indexed [x, y, ...]; natural order has x fastest
    return np.transpose(out).reshape(-1)


# -------------------------------------------------------------- dispatcher
def oracle_diag(dims, d, t, method="auto"):
    """diag(H^{-1}) for every frequency row of d [K,N] (open boundaries)."""
    d = np.atleast_2d(np.asarray(d, dtype=np.complex128))
    n = d.shape[1]
    if method == "auto":
        method = "dense" if n <= 1600 else "rgf"
    f = diag_inv_dense if method == "dense" else diag_inv_rgf
    return np.stack([f(dims, d[k], t) for k in range(d.shape[0])])


def rel_err(G, G_ref):
    """Componentwise relative error max |G - G_ref| / |G_ref| (the accuracy
    measure used for every comparison; |G_ii| > 0 whenever Im H > 0)."""
    G = np.asarray(G)
    G_ref = np.asarray(G_ref)
    return float(np.max(np.abs(G - G_ref) / np.abs(G_ref)))
