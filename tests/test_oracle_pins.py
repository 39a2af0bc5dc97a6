"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-type the oracle's own formulas: each compares two different
routes to the same number (closed forms, continued fractions, an independent
algorithm, invariances) or checks a structural fact the paper states.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import dyson as od
from oracle import lowrank as olr

HERE = os.path.dirname(os.path.abspath(__file__))


def _rand_d(n, omega=0.4, seed=0, mu=0.3):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0, 1, n)
    b = rng.uniform(-0.5, 0.5, n)
    V = rng.uniform(0, 2, n)
    sig = a / (1j * omega + b)
    return oracle.assemble_diag(V, [omega], sig[None, :], mu)[0]


# ---------------------------------------------------------------- P1 / P2
@pytest.mark.parametrize("dims", [(7,), (6, 5), (5, 3), (4, 3, 5), (3, 3, 3)])
@pytest.mark.parametrize("t", [-1.0, 0.7])
def test_periodic_closed_form(dims, t):
    """Uniform periodic lattice, V = Sigma = 0: G_ii = (1/N) sum_k 1/(iw+mu+2t sum cos k)."""
    n = int(np.prod(dims))
    omega, mu = 0.37, 0.5
    V = np.zeros(n)
    sig = np.zeros((1, n), dtype=complex)
    d = oracle.assemble_diag(V, [omega], sig, mu)[0]
    G = od.diag_inv_dense(dims, d, t, periodic=True)
    ref = oracle.closed_form_periodic(dims, 1j * omega + mu, t)
    assert np.max(np.abs(G - ref)) / abs(ref) < 1e-13


@pytest.mark.parametrize("dims", [(9,), (6, 5), (4, 3, 5)])
def test_open_uniform_closed_form(dims):
    """Uniform open lattice: sine-mode expansion equals O1 and O2."""
    n = int(np.prod(dims))
    z = 0.2 + 0.31j
    d = np.full(n, z)
    ref = oracle.closed_form_open_uniform(dims, z, -1.0)
    assert oracle.rel_err(od.diag_inv_dense(dims, d, -1.0), ref) < 1e-13
    assert oracle.rel_err(od.diag_inv_rgf(dims, d, -1.0), ref) < 1e-13


@pytest.mark.parametrize("dims", [(9,), (6, 5), (4, 3, 5)])
@pytest.mark.parametrize("c", [0.7, -1.3])
def test_potential_enters_with_minus_sign(dims, c):
    """eq. (1) subtracts V_i: a uniform potential V_i = c with Sigma = 0 is
    the uniform open lattice at the shifted energy z = i w + mu - c, whose
    sine-mode closed form is independent of the assembly.  A planted +V
    (the closed form at i w + mu + c) fails the same comparison."""
    n = int(np.prod(dims))
    om, mu, t = np.array([0.37]), 0.4, -1.0
    V = np.full(n, c)
    sig = np.zeros((1, n), complex)
    d = oracle.assemble_diag(V, om, sig, mu)[0]
    ref = oracle.closed_form_open_uniform(dims, 1j * om[0] + mu - c, t)
    assert oracle.rel_err(od.diag_inv_dense(dims, d, t), ref) < 1e-13
    assert oracle.rel_err(od.diag_inv_rgf(dims, d, t), ref) < 1e-13
    planted = (1j * om[0] + mu) + V - sig[0]
    assert oracle.rel_err(od.diag_inv_dense(dims, planted, t), ref) > 1e-2


def test_site_potential_shifts_only_its_site_at_high_frequency():
    """A potential on one site: to first order in 1/|d| the change of G_jj is
    -(1/(z - V_j) - 1/z) on that site only, with the sign of -V_j fixed by
    eq. (1) (z = i w + mu, uniform elsewhere, t small against |z|)."""
    dims, n = (5, 4), 20
    om, mu, t, j, vj = np.array([30.0]), 0.2, -0.05, 7, 2.5
    V = np.zeros(n)
    V[j] = vj
    d = oracle.assemble_diag(V, om, np.zeros((1, n), complex), mu)[0]
    G = od.diag_inv_dense(dims, d, t)
    z = 1j * om[0] + mu
    assert abs(G[j] - 1.0 / (z - vj)) < 10 * t * t / abs(z) ** 3
    assert abs(G[j] - 1.0 / (z + vj)) > 100 * t * t / abs(z) ** 3
    others = np.delete(np.arange(n), j)
    assert np.max(np.abs(G[others] - 1.0 / z)) < 10 * t * t / abs(z) ** 3


@pytest.mark.parametrize("dims,per", [((6, 5), (1, 0)), ((5, 7), (0, 1)), ((4, 3, 5), (0, 1, 1)),
                                      ((3, 4, 3), (1, 0, 1)), ((8,), (1,))])
def test_mixed_boundary_closed_form(dims, per):
    """Uniform lattice with some axes periodic: the product-of-chain-modes
    closed form equals O1 with per-axis wrap bonds; a wrong axis flag fails."""
    n = int(np.prod(dims))
    z = 0.35 + 0.29j
    d = np.full(n, z)
    ref = oracle.closed_form_uniform(dims, z, -1.0, per)
    assert oracle.rel_err(od.diag_inv_dense(dims, d, -1.0, periodic=per), ref) < 1e-12
    wrong = tuple(1 - p for p in per)
    assert oracle.rel_err(od.diag_inv_dense(dims, d, -1.0, periodic=wrong), ref) > 1e-3


def test_uniform_closed_form_reduces_to_the_pure_cases():
    """All axes periodic or all open: the mixed closed form gives the same
    numbers as the two separate closed forms."""
    dims, z = (5, 4, 3), 0.1 + 0.4j
    G = oracle.closed_form_uniform(dims, z, 0.8, (1, 1, 1))
    assert np.max(np.abs(G - oracle.closed_form_periodic(dims, z, 0.8))) < 1e-13
    G = oracle.closed_form_uniform(dims, z, 0.8, (0, 0, 0))
    assert oracle.rel_err(G, oracle.closed_form_open_uniform(dims, z, 0.8)) < 1e-13


def test_complex_energy_assembly():
    """eq. (1) at z = i w is the Matsubara assembly; at a real-axis energy the
    dense inverse of a uniform periodic lattice meets the plane-wave closed
    form, and Im G < 0 (retarded)."""
    dims = (6, 5)
    n = 30
    rng = np.random.default_rng(4)
    V = rng.uniform(0, 1, n)
    om = np.array([0.3, 1.1])
    sig = rng.uniform(-0.2, 0.2, (2, n)) + 1j * rng.uniform(-0.2, 0.0, (2, n))
    assert np.array_equal(oracle.assemble_diag_z(V, 1j * om, sig, 0.4),
                          oracle.assemble_diag(V, om, sig, 0.4))
    z = np.array([-0.7 + 0.05j])
    d = oracle.assemble_diag_z(np.zeros(n), z, np.zeros((1, n)), 0.5)[0]
    G = od.diag_inv_dense(dims, d, -1.0, periodic=True)
    ref = oracle.closed_form_periodic(dims, z[0] + 0.5, -1.0)
    assert np.max(np.abs(G - ref)) / abs(ref) < 1e-12
    assert np.all(G.imag < 0)


def test_odd_periodic_sees_hopping_sign():
    """On a non-bipartite (odd periodic) lattice the sign of t is observable:
    the oracle must follow H_ij = +t (eq. (1)), not -t."""
    dims = (5, 3)
    n = 15
    z = 0.5 + 0.37j
    G = od.diag_inv_dense(dims, np.full(n, z), -1.0, periodic=True)
    assert abs(G[0] - oracle.closed_form_periodic(dims, z, -1.0)) < 1e-13
    assert abs(G[0] - oracle.closed_form_periodic(dims, z, +1.0)) > 1e-3


# ---------------------------------------------------------------- P3 / P4 / P5
def test_inverse_is_symmetric():
    dims = (6, 7)
    d = _rand_d(42, seed=3)
    Gf = od.diag_inv_dense(dims, d, -1.0, full=True)
    assert np.max(np.abs(Gf - Gf.T)) < 1e-13 * np.max(np.abs(Gf))
    # and it is not Hermitian: the conjugate transpose differs
    assert np.max(np.abs(Gf - Gf.conj().T)) > 1e-3


def test_bipartite_gauge():
    """Open square lattices are bipartite: G_ii(t) = G_ii(-t)."""
    dims = (6, 5)
    d = _rand_d(30, seed=4)
    assert oracle.rel_err(od.diag_inv_dense(dims, d, 1.0), od.diag_inv_dense(dims, d, -1.0)) < 1e-12


def test_zero_hopping():
    dims = (4, 5)
    d = _rand_d(20, seed=5)
    assert oracle.rel_err(od.diag_inv_dense(dims, d, 0.0), 1.0 / d) < 1e-15
    assert oracle.rel_err(od.diag_inv_rgf(dims, d, 0.0), 1.0 / d) < 1e-15


# ---------------------------------------------------------------- P6
def _chain_continued_fraction(d, t):
    n = len(d)
    gl = np.zeros(n, complex)
    gr = np.zeros(n, complex)
    for i in range(n):
        gl[i] = 1.0 / (d[i] - (t * t * gl[i - 1] if i else 0.0))
    for i in range(n - 1, -1, -1):
        gr[i] = 1.0 / (d[i] - (t * t * gr[i + 1] if i < n - 1 else 0.0))
    out = np.empty(n, complex)
    for i in range(n):
        s = d[i]
        if i:
            s -= t * t * gl[i - 1]
        if i < n - 1:
            s -= t * t * gr[i + 1]
        out[i] = 1.0 / s
    return out


def test_chain_continued_fraction():
    d = _rand_d(23, seed=6)
    ref = _chain_continued_fraction(d, -1.0)
    assert oracle.rel_err(od.diag_inv_dense((23,), d, -1.0), ref) < 1e-12
    assert oracle.rel_err(od.diag_inv_rgf((23,), d, -1.0), ref) < 1e-12


# ---------------------------------------------------------------- P7 / P8
def test_causality_bounds():
    """Im H = diag(w + Im(-Sigma)) > 0 for a causal Sigma, hence Im G_ii < 0
    and |G_ii| <= 1 / min_i Im H_ii."""
    w = synth.scaled_square(20, 3)
    V, om, sig = synth.make_inputs(w)
    d = oracle.assemble_diag(V, om, sig, w.mu)
    assert np.all(d.imag >= om[:, None] - 1e-15)
    for k in range(3):
        G = od.diag_inv_dense(w.dims, d[k], w.t)
        assert np.all(G.imag < 0)
        assert np.max(np.abs(G)) <= 1.0 / np.min(d[k].imag) * (1 + 1e-12)


def test_sigma_sign_is_subtracted():
    """a=1, b=0: Sigma = -i/w, so -Sigma adds +i/w to Im H; with the opposite
    sign Im H_ii = w - 1/w < 0 for w < 1 and causality would fail."""
    om = np.array([0.5])
    sig = np.full((1, 4), 1.0 / (1j * 0.5))
    d = oracle.assemble_diag(np.zeros(4), om, sig, 0.0)
    assert np.allclose(d.imag, 0.5 + 2.0)


def test_high_frequency_expansion():
    """For |d| >> |t|: G_ii = 1/d_i + sum_{j~i} t^2/(d_i^2 d_j) + O(Z^2 t^4/|d|^5)."""
    dims = (5, 4)
    n = 20
    rng = np.random.default_rng(8)
    d = 40j + rng.uniform(-1, 1, n) + 1j * rng.uniform(0, 1, n)
    G = od.diag_inv_dense(dims, d, -1.0)
    r, c = od._bonds(dims)
    second = np.zeros(n, complex)
    np.add.at(second, r, 1.0 / (d[r] ** 2 * d[c]))
    np.add.at(second, c, 1.0 / (d[c] ** 2 * d[r]))
    approx = 1.0 / d + second
    # closed 4-step walks on the square lattice number at most 36
    assert np.max(np.abs(G - approx)) < 40.0 / np.min(np.abs(d)) ** 5
    # the t^2 term matters at this order: dropping it is detectably worse
    assert np.max(np.abs(G - 1.0 / d)) > 10 * np.max(np.abs(G - approx))


# ---------------------------------------------------------------- P12
@pytest.mark.parametrize("dims", [(13, 11), (6, 5, 4)])
def test_three_oracle_tiers_agree(dims):
    n = int(np.prod(dims))
    d = _rand_d(n, seed=9)
    G1 = od.diag_inv_dense(dims, d, -1.0)
    G2 = od.diag_inv_rgf(dims, d, -1.0)
    sites = [0, 1, n // 2, n - 1]
    G3 = od.diag_inv_sampled(dims, d, -1.0, sites)
    assert oracle.rel_err(G2, G1) < 1e-12
    assert oracle.rel_err(G3, G1[sites]) < 1e-12
    every = np.arange(n)
    G3nd = od.diag_inv_sampled(dims, d, -1.0, every, order="nd")
    assert oracle.rel_err(G3nd, G1) < 1e-12


@pytest.mark.parametrize("dims", [(13, 11), (9, 8, 7), (20,), (5, 9, 6)])
def test_nested_dissection_order_is_a_permutation(dims):
    """The relabelling O3 may factor with visits every site exactly once."""
    p = od.nested_dissection_order(dims)
    assert np.array_equal(np.sort(p), np.arange(int(np.prod(dims))))


# ---------------------------------------------------------------- P11 (Fig. 1)
def test_fig1_structure():
    g = json.load(open(os.path.join(HERE, "golden", "fig1_dd_example.json")))
    dims = tuple(g["lattice"])
    nodes = olr.plan_boxes(dims, 3, "single")
    root = nodes[0]
    leaves = [nd for nd in nodes if not nd["splits"]]
    assert len(leaves) == g["n_subdomains"]
    mask = olr._interface_mask(dims, root["box"], root["splits"])
    assert int(mask.sum()) == g["m"]
    assert g["N"] - int(mask.sum()) == g["interface_labels_first"] - 1
    assert g["interface_labels_last"] - g["interface_labels_first"] + 1 == g["m"]
    # the method is exact after about m steps (m + 1 with a random start)
    d = _rand_d(25, seed=11)
    G, info = oracle.lowrank_diag(dims, d, -1.0, 3, "single", return_info=True)
    assert info[0]["m"] == g["m"]
    assert info[0]["steps"] <= g["lanczos_steps_needed"] + 2
    assert oracle.rel_err(G, od.diag_inv_dense(dims, d, -1.0)) < 1e-11


# ---------------------------------------------------------------- P9 / P10 / P13
def test_lowrank_full_rank_matches_oracle_small32():
    """The spec check: the low-rank method at full interface rank equals
    the plain definition (eqs. (8)-(9) make it exact)."""
    w = synth.SMALL_32
    V, om, sig = synth.make_inputs(w)
    d = oracle.assemble_diag(V, om, sig, w.mu)[0]
    ref = od.diag_inv_dense(w.dims, d, w.t)
    G, info = oracle.lowrank_diag(w.dims, d, w.t, 16, "single", return_info=True)
    assert info[0]["m"] == 63
    assert oracle.rel_err(G, ref) < 1e-10
    Gn = oracle.lowrank_diag(w.dims, d, w.t, 16, "nested")
    assert oracle.rel_err(Gn, ref) < 1e-10


def test_lowrank_invariant_to_partition_and_seed():
    dims = (21, 18)
    d = _rand_d(21 * 18, seed=12)
    ref = od.diag_inv_dense(dims, d, -1.0)
    for s, part, seed in [(8, "single", 0), (8, "nested", 1), (5, "nested", 2), (11, "single", 3)]:
        G = oracle.lowrank_diag(dims, d, -1.0, s, part, seed=seed)
        assert oracle.rel_err(G, ref) < 1e-10, (s, part, seed)


def test_explicit_schur_equals_lowrank_form():
    """eq. (6): H^{-1} = blkdiag(B^{-1},0) + W S^{-1} W^T with W = [B^{-1}E; -I]
    and S = C - E^T B^{-1} E (eq. (5)); X of eq. (7) has rank m."""
    dims = (7, 7)
    d = _rand_d(49, seed=13)
    H = od.dense_hamiltonian(dims, d, -1.0)
    nodes = olr.plan_boxes(dims, 4, "single")
    mask = olr._interface_mask(dims, nodes[0]["box"], nodes[0]["splits"])
    ib, ic = np.where(~mask)[0], np.where(mask)[0]
    B, E, C = H[np.ix_(ib, ib)], H[np.ix_(ib, ic)], H[np.ix_(ic, ic)]
    Binv = np.linalg.inv(B)
    S = C - E.T @ Binv @ E
    W = np.vstack([Binv @ E, -np.eye(len(ic))])
    X = W @ np.linalg.inv(S) @ W.T
    Hinv = np.zeros_like(H)
    perm = np.concatenate([ib, ic])
    Hinv[np.ix_(perm, perm)] = X
    Hinv[np.ix_(ib, ib)] += Binv
    assert np.max(np.abs(Hinv - np.linalg.inv(H))) < 1e-12
    assert np.linalg.matrix_rank(X, tol=1e-10) == len(ic)


def test_truncated_rank_is_not_exact():
    """Rank k < m leaves an O(1)-scale error (finding behind the full-rank
    requirement); full rank removes it."""
    w = synth.SMALL_32
    V, om, sig = synth.make_inputs(w)
    d = oracle.assemble_diag(V, om, sig, w.mu)[0]
    ref = od.diag_inv_dense(w.dims, d, w.t)
    e_half = oracle.rel_err(oracle.lowrank_diag(w.dims, d, w.t, 16, "single", max_rank=32), ref)
    assert e_half > 1e-3


# ---------------------------------------------------------------- planted mistakes
def _lanczos_conjugated(xmatvec, q1, kmax, tol):
    """A plausible mistake: Hermitian (conjugating) products instead of the
    bilinear ones of Sec. II.A."""
    n = q1.shape[0]
    q = q1 / np.sqrt(np.vdot(q1, q1))
    q_prev = np.zeros(n, complex); beta = 0.0; Q = []; D = np.zeros(n, complex)
    for j in range(kmax):
        Q.append(q); u = xmatvec(q); alpha = np.vdot(q, u)
        r = u - alpha * q - beta * q_prev
        Qm = np.array(Q)
        for _ in range(2):
            r = r - Qm.T @ (Qm.conj() @ r)
        D += alpha * q * q
        if j > 0:
            D += 2 * beta * q_prev * q
        if np.linalg.norm(r) <= tol * np.linalg.norm(u):
            break
        beta = np.sqrt(np.vdot(r, r)); q_prev, q = q, r / beta
    return D, j + 1, None, None


def _lanczos_no_beta(xmatvec, q1, kmax, tol):
    """A plausible mistake: only the alpha_j q_j*q_j terms of the three-vector
    diagonal formula, dropping the beta terms of T."""
    n = q1.shape[0]
    q = q1 / np.sqrt(q1 @ q1); q_prev = np.zeros(n, complex); beta = 0.0; Q = []
    D = np.zeros(n, complex)
    for j in range(kmax):
        Q.append(q); u = xmatvec(q); alpha = q @ u
        r = u - alpha * q - beta * q_prev
        Qm = np.array(Q)
        for _ in range(2):
            r = r - Qm.T @ (Qm @ r)
        D += alpha * q * q
        if np.linalg.norm(r) <= tol * np.linalg.norm(u):
            break
        beta = np.sqrt(r @ r); q_prev, q = q, r / beta
    return D, j + 1, None, None


@pytest.mark.parametrize("planted", [_lanczos_conjugated, _lanczos_no_beta])
def test_pin_rejects_planted_lanczos_mistakes(monkeypatch, planted):
    dims = (12, 12)
    d = _rand_d(144, seed=14)
    ref = od.diag_inv_dense(dims, d, -1.0)
    monkeypatch.setattr(olr, "bilinear_lanczos_diag", planted)
    G = oracle.lowrank_diag(dims, d, -1.0, 6, "single")
    assert oracle.rel_err(G, ref) > 1e-4


def test_pin_rejects_planted_rgf_mistake(monkeypatch):
    """The slice recursion with t instead of t^2 (a dropped factor) must fail
    the O1 = O2 pin."""
    dims = (6, 7)
    d = _rand_d(42, seed=15)
    ref = od.diag_inv_dense(dims, d, -1.5)
    assert oracle.rel_err(od.diag_inv_rgf(dims, d, -1.5), ref) < 1e-12
    real_inv = np.linalg.inv
    G_ok = od.diag_inv_rgf(dims, d, -1.5)
    # plant the slip directly: a copy of the recursion with the wrong power
    D = d.reshape(7, 6)
    r, c = od._bonds((6,))
    T = np.zeros((6, 6), complex); T[r, c] = -1.5; T[c, r] = -1.5
    g, prev = [], None
    for s_ in range(7):
        A = T + np.diag(D[s_])
        if prev is not None:
            A = A - (-1.5) * prev               # planted: t instead of t^2
        prev = real_inv(A); g.append(prev)
    out = [np.diag(g[-1])]
    Gss = g[-1]
    for s_ in range(5, -1, -1):
        Gss = g[s_] + 2.25 * (g[s_] @ Gss @ g[s_]); out.append(np.diag(Gss))
    bad = np.concatenate(out[::-1])
    assert oracle.rel_err(G_ok, ref) < 1e-12
    assert oracle.rel_err(bad, ref) > 1e-3


def test_interface_space_lanczos_over_start_vectors():
    """Lanczos on the Schur complement (interface space, one subdomain solve per
    step, H^{-1} of the projected Hessenberg matrix) reproduces diag(H^{-1}) at
    full interface rank for every one of 40 start vectors on the 32x32 one-level
    decomposition (m = 63), and for a recursive one; its accuracy depends on the
    start vector more than the X form's (median and worst case recorded)."""
    w = synth.SMALL_32
    V, om, sig = synth.make_inputs(w)
    d = oracle.assemble_diag(V, om, sig, w.mu)[0]
    ref = od.diag_inv_dense(w.dims, d, w.t)
    errs = [oracle.rel_err(olr.interface_lanczos_diag(w.dims, d, w.t, 16, "single", seed=k), ref)
            for k in range(40)]
    print(f"interface Lanczos, 40 start vectors: median {np.median(errs):.2e}, max {max(errs):.2e}")
    assert max(errs) < 1e-9 and np.median(errs) < 1e-11
    dims = (37, 29)
    d2 = _rand_d(37 * 29, seed=21)
    G2 = olr.interface_lanczos_diag(dims, d2, -1.0, 8, "nested", seed=3)
    assert oracle.rel_err(G2, od.diag_inv_dense(dims, d2, -1.0)) < 1e-9
