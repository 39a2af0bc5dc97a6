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
