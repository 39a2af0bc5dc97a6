"""Helpers shared by the GPU tests: seeded inputs on the device and the
oracle's answer for them (computed on the CPU from the same arrays)."""
import numpy as np

import oracle
import synth


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def device_inputs(w):
    import torch
    V, om, sig = synth.make_inputs(w)
    dev = torch.device("cuda:0")
    return (V, om, sig,
            torch.from_numpy(V).to(dev), torch.from_numpy(om).to(dev),
            torch.from_numpy(np.ascontiguousarray(sig)).to(dev))


def oracle_G(w, V, om, sig, method="auto", freqs=None):
    d = oracle.assemble_diag(V, om, sig, w.mu)
    if freqs is not None:
        d = d[list(freqs)]
    return oracle.oracle_diag(w.dims, d, w.t, method=method)


def leaf_oracle(w, d_row, plan):
    """diag(B_s^{-1}) per leaf (dense inverse of the lattice restricted to
    the leaf's sites), 0 on separator sites; plan maps from the library."""
    depth, is_sep, tile = plan.maps()
    n = w.n_sites
    H = oracle.dense_hamiltonian(w.dims, d_row, w.t)
    out = np.zeros(n, complex)
    for tt in np.unique(tile[is_sep == 0]):
        idx = np.where((tile == tt) & (is_sep == 0))[0]
        out[idx] = np.diag(np.linalg.inv(H[np.ix_(idx, idx)]))
    return out


def o3_nd_sites(args):
    """Worker: O3 (sparse LU of the nested-dissection relabelling, unit solves)
    at the given sites of one frequency; prints each step as it finishes."""
    import sys
    import time
    import scipy.sparse.linalg as spla
    from oracle import dyson as od
    dims, d_row, t, sites, tag = args
    t0 = time.perf_counter()
    H = od.hamiltonian(dims, d_row, t)
    n = H.shape[0]
    perm = od.nested_dissection_order(dims)
    where = np.empty_like(perm)
    where[perm] = np.arange(n)
    lu = spla.splu(H[perm][:, perm].tocsc(), permc_spec="NATURAL", diag_pivot_thresh=0.0)
    print(f"O3 {tag}: factored in {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    rows = where[np.asarray(sites)]
    out = np.empty(len(rows), dtype=np.complex128)
    for c0 in range(0, len(rows), 32):
        r = rows[c0:c0 + 32]
        E = np.zeros((n, len(r)), dtype=np.complex128)
        E[r, np.arange(len(r))] = 1.0
        out[c0:c0 + len(r)] = lu.solve(E)[r, np.arange(len(r))]
        print(f"O3 {tag}: {c0 + len(r)}/{len(rows)} sites, {time.perf_counter() - t0:.0f} s",
              file=sys.stderr, flush=True)
    return out
