"""GPU parity tests: each stage of the hot path and the full solve, called
through the C ABI, against the CPU oracle on the same seeded inputs.

Tolerances (componentwise relative error unless noted):
  assembly                1e-15  (same three operations in FP64)
  leaf diag(B^{-1})       1e-12  (pivot-free block LDL^T, |growth| ~ 2)
  X-matvec                1e-10 of max|u| (inner COCG to 1e-13 relative)
  full solve, FP64        1e-10  (full interface rank; the bilinear Lanczos
                                  in FP64 lands at 1e-13..1e-11 here)
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import device_inputs, oracle_G, leaf_oracle, have_gpu

pytestmark = pytest.mark.gpu

if have_gpu():
    import torch
    from paper_1102_3137_amd import (Plan, PART_NESTED, PART_SINGLE, PREC_FP64, PREC_MIXED,
                                     PREC_MIXED16, DysonError)


def _plan(w, s=16, part=0, prec=0, **kw):
    return Plan(w.dims, t=w.t, mu=w.mu, leaf_edge=s, partition=part, precision=prec, **kw)


def _case(dims, K=2, seed=7, vc=None, beta=10.0, mu=0.5):
    if vc is None:
        vc = 0.01 * (32.0 / max(dims)) ** 2
    return synth.rect(dims, K=K, seed=seed, vc=vc, mu=mu, beta=beta)


def test_assemble_eq1():
    w = _case((37, 29), K=3)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 8)
    d = p.assemble(tV, tom, tsig).cpu().numpy()
    ref = oracle.assemble_diag(V, om, sig, w.mu)
    assert oracle.rel_err(d, ref) <= 1e-15


@pytest.mark.parametrize("dims,s", [((32, 32), 16), ((37, 29), 8), ((5, 5), 3), ((40,), 8), ((16, 16), 16),
                                    ((9, 8, 7), 4), ((12, 12, 12), 6)])
def test_leaf_diag(dims, s):
    w = _case(dims, K=2)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, s)
    d = p.assemble(tV, tom, tsig)
    G = p.leaf_diag(d).cpu().numpy()
    dn = d.cpu().numpy()
    for k in range(w.n_freq):
        ref = leaf_oracle(w, dn[k], p)
        leaf = ref != 0
        assert np.all(G[k][~leaf] == 0)
        assert oracle.rel_err(G[k][leaf], ref[leaf]) < 1e-12


def _dense_X_apply(w, d_row, p, level, q):
    """u = X q for every domain of the level, X = H_D^{-1} - blkdiag(B_D^{-1}, 0)
    with H_D the lattice on the domain's sites and B_D its sites deeper than
    the level (dense, from the oracle's H)."""
    depth, is_sep, tile = p.maps()
    H = oracle.dense_hamiltonian(w.dims, d_row, w.t)
    n = w.n_sites
    u = np.zeros(n, complex)
    # sites of the level's domains: not a separator of a shallower level and
    # (for leaves) not a leaf shallower than or at the level
    act = np.where(is_sep == 1, depth >= level, depth > level)
    # connected components of act under the lattice bonds are the domains
    import scipy.sparse.csgraph as cg
    import scipy.sparse as sps
    idx = np.where(act)[0]
    A = (np.abs(H[np.ix_(idx, idx)]) > 0).astype(float)
    ncomp, lab = cg.connected_components(sps.csr_matrix(A), directed=False)
    for c in range(ncomp):
        dom = idx[lab == c]
        sepc = (is_sep[dom] == 1) & (depth[dom] == level)
        if not sepc.any():
            continue
        Hd = H[np.ix_(dom, dom)]
        X = np.linalg.inv(Hd)
        b = dom[~sepc]
        bi = np.where(~sepc)[0]
        X[np.ix_(bi, bi)] -= np.linalg.inv(H[np.ix_(b, b)])
        u[dom] = X @ q[dom]
    return u


# tile shapes for the inner-solve kernels' halo slots (2 D s^(D-1) per tile):
# 64 (16^2), 32 (8^2), 48 (12^2, 144 sites), 2 (chains), 96 (4^3, two slots
# per lane), 54 (3^3), 24 (2^3), and the workgroup kernels' 150 (5^3), 216 (6^3)
@pytest.mark.parametrize("dims,s,part", [((32, 32), 16, 0), ((32, 32), 16, 1), ((37, 29), 8, 0),
                                         ((5, 5), 3, 1), ((40,), 8, 0), ((9, 8, 7), 4, 0),
                                         ((11, 9, 7), 4, 1), ((12, 11, 10), 6, 0),
                                         ((11, 10, 9), 5, 1), ((36, 26), 12, 0), ((50,), 16, 0),
                                         ((7, 6, 5), 3, 0), ((6, 5, 6), 2, 1)])
def test_xmatvec(dims, s, part):
    w = _case(dims, K=2)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, s, part)
    d = p.assemble(tV, tom, tsig)
    dn = d.cpu().numpy()
    rng = np.random.default_rng(3)
    q = rng.standard_normal((w.n_freq, w.n_sites)) + 1j * rng.standard_normal((w.n_freq, w.n_sites))
    tq = torch.from_numpy(q).cuda()
    for level in range(p.info.levels):
        u = p.xmatvec(level, d, tq).cpu().numpy()
        for k in range(w.n_freq):
            ref = _dense_X_apply(w, dn[k], p, level, q[k])
            assert np.max(np.abs(u[k] - ref)) <= 1e-10 * np.max(np.abs(ref)), (level, k)


@pytest.mark.parametrize("dims,s,part", [((32, 32), 16, 1), ((37, 29), 8, 0), ((9, 8, 7), 4, 0)])
def test_correct_level_matches_dense_diag_X(dims, s, part):
    """One level of bilinear Lanczos with the streaming diagonal: the added
    diag(Q T Q^T) equals diag(X) of every domain of the level."""
    w = _case(dims, K=2)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, s, part)
    d = p.assemble(tV, tom, tsig)
    dn = d.cpu().numpy()
    depth, is_sep, tile = p.maps()
    H = [oracle.dense_hamiltonian(w.dims, dn[k], w.t) for k in range(w.n_freq)]
    for level in range(p.info.levels):
        G0 = torch.zeros_like(d)
        steps = p.correct_level(level, d, G0)
        D = G0.cpu().numpy()
        for k in range(w.n_freq):
            Xd = _dense_X_diag(w, H[k], depth, is_sep, level)
            assert np.max(np.abs(D[k] - Xd)) <= 1e-10 * np.max(np.abs(Xd)), (level, k)
        # full rank: X of a domain has rank m (eq. (7)), so every (domain,
        # frequency) took at least m steps, and no more than its step cap
        m, cap = p.domains(level)
        assert steps.shape == (w.n_freq, len(m))
        assert np.all(steps >= m[None, :]), (level, steps, m)
        assert np.all(steps <= cap[None, :]), (level, steps, cap)


def _dense_X_diag(w, H, depth, is_sep, level):
    import scipy.sparse.csgraph as cg
    import scipy.sparse as sps
    act = np.where(is_sep == 1, depth >= level, depth > level)
    idx = np.where(act)[0]
    A = (np.abs(H[np.ix_(idx, idx)]) > 0).astype(float)
    ncomp, lab = cg.connected_components(sps.csr_matrix(A), directed=False)
    out = np.zeros(w.n_sites, complex)
    for c in range(ncomp):
        dom = idx[lab == c]
        sepc = (is_sep[dom] == 1) & (depth[dom] == level)
        if not sepc.any():
            continue
        X = np.linalg.inv(H[np.ix_(dom, dom)])
        bi = np.where(~sepc)[0]
        X[np.ix_(bi, bi)] -= np.linalg.inv(H[np.ix_(dom[bi], dom[bi])])
        out[dom] = np.diag(X)
    return out


SOLVE_CASES = [
    (synth.SMALL_32, 16, 1),                     # 4 subdomains of 16x16, one level, m = 63
    (synth.SMALL_32, 16, 0),                     # recursive bisection
    (_case((37, 29), K=3), 8, 0),                # ragged tiles, several levels
    (_case((5, 5), K=2), 3, 1),                  # Fig. 1 layout, m = 9
    (_case((40,), K=2), 8, 0),                   # chain
    (_case((16, 16), K=2), 16, 0),               # a single leaf: no correction level
    (_case((48, 33), K=4, beta=20.0), 16, 0),    # more frequencies, uneven halves
    (_case((9, 8, 7), K=2, mu=1.0), 4, 0),       # cubic lattice (Z = 6), ragged tiles
    (_case((11, 9, 7), K=2, mu=1.0), 4, 1),      # cubic, one level
    (_case((12, 12, 12), K=3, mu=1.0, beta=10.0), 6, 0),  # cubic, 6^3 tiles
    (_case((13, 11, 10), K=2, mu=1.0), 5, 0),    # cubic, 5^3 tiles (25-site planes), ragged
]


@pytest.mark.parametrize("w,s,part", SOLVE_CASES, ids=[f"{c[0].dims}-s{c[1]}-p{c[2]}" for c in SOLVE_CASES])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "mixed", "mixed16"])
def test_solve_full_rank(w, s, part, prec):
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, s, part, prec)
    G, rep = p.solve(tV, tom, tsig, report=True)
    ref = oracle_G(w, V, om, sig)
    err = oracle.rel_err(G.cpu().numpy(), ref)
    print(f"{w.dims} s={s} part={part} prec={prec} err={err:.2e} rep={rep}")
    assert err < 1e-10
    assert rep["truncated"] == 0      # every domain reached exhaustion


def test_batch_invariance_and_determinism():
    """Each frequency's result is the same computed alone or in the batch,
    bit for bit, and a repeated solve is bitwise identical."""
    w = _case((37, 29), K=4, beta=20.0)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 8)
    G1 = p.solve(tV, tom, tsig).cpu().numpy()
    G2 = p.solve(tV, tom, tsig).cpu().numpy()
    assert np.array_equal(G1, G2)
    for k in [0, 3]:
        Gk = p.solve(tV, tom[k:k + 1].contiguous(), tsig[k:k + 1].contiguous()).cpu().numpy()
        assert np.array_equal(Gk[0], G1[k])


def test_truncated_rank_reports_and_errs():
    w = synth.SMALL_32
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 16, 1, max_rank=32)
    G, rep = p.solve(tV, tom, tsig, report=True)
    err = oracle.rel_err(G.cpu().numpy(), oracle_G(w, V, om, sig))
    assert rep["truncated"] == 1 and rep["max_rank_used"] <= 32
    assert err > 1e-3     # rank 32 < m = 63 is not exact


def test_invalid_inputs_rejected():
    w = _case((20, 20), K=2)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 8)
    bad = tom.clone()
    bad[1] = -0.1
    with pytest.raises(DysonError) as e:
        p.solve(tV, bad, tsig)
    assert e.value.status == 1
    sig2 = tsig.clone()
    sig2[0, 5] = complex(0.0, 5.0)      # Im Sigma > w: not causal
    with pytest.raises(DysonError) as e:
        p.solve(tV, tom, sig2)
    assert e.value.status == 1
    # more frequencies in one call than the launch grid holds: refused up front
    from paper_1102_3137_amd import binding as B
    assert B.load_library().dyson_solve(p.plan, 70000, None, None, None, None, None,
                                        None) == 1


@pytest.mark.parametrize("L,freqs,prec", [(128, (0, 1, 31, 63), 1), (128, (0, 63), 0),
                                          (128, (0, 63), 2), (256, (0, 63), 1),
                                          (256, (0, 31, 63), 0)])
def test_solve_large_lattice(L, freqs, prec):
    """Recursive bisection with 16x16 tiles at 128^2 (6 levels) and 256^2
    (8 levels, the throughput workload's lattice) on the hardest and easiest
    Matsubara frequencies, against the block-tridiagonal oracle, at the library
    defaults (inner solves to 1e-14, Lanczos 1e-11): 1e-10 in every
    precision (the mixed preconditioners change the iteration counts, the
    residuals and the Lanczos run stay FP64)."""
    w = synth.Workload(dims=(L, L), t=-1.0, mu=0.5, vc=2e-4 * (256.0 / L) ** 2, beta=20.0,
                       freq_index=tuple(freqs), seed=2, name=f"square {L}")
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 16, 0, prec)
    G, rep = p.solve(tV, tom, tsig, report=True)
    ref = oracle_G(w, V, om, sig, method="rgf")
    err = oracle.rel_err(G.cpu().numpy(), ref)
    print(f"{L}^2 freqs={freqs} prec={prec} err={err:.2e} rep={rep}")
    assert rep["truncated"] == 0 and rep["capped_items"] == 0
    assert err < 1e-10


def test_bench_configuration_256():
    """The throughput workload exactly as the benchmark runs it: 256^2, 16x16
    tiles, recursive bisection, complex32 preconditioner factors, inner solves
    to 1e-11, Lanczos 1e-11, six concurrent level groups; frequencies
    w_0, w_31 and w_63 of the beta = 20 grid, every site against the
    block-tridiagonal oracle.  The metric counts results within 1e-6; at
    this inner tolerance the method lands near 1e-9, asserted below the
    paper's one part in 1e8."""
    w = synth.Workload(dims=(256, 256), t=-1.0, mu=0.5, vc=2e-4, beta=20.0,
                       freq_index=(0, 31, 63), seed=2, name="square 256")
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 16, 0, PREC_MIXED16, inner_tol=1e-11, lanczos_tol=1e-11, level_streams=6)
    G, rep = p.solve(tV, tom, tsig, report=True)
    err = oracle.rel_err(G.cpu().numpy(), oracle_G(w, V, om, sig, method="rgf"))
    print(f"bench configuration err={err:.2e} rep={rep}")
    assert rep["truncated"] == 0 and rep["capped_items"] == 0
    assert err < 1e-8
    assert 0 < rep["est_rel_err"] < 1e-8


def test_loose_lanczos_tolerance_stays_accurate():
    """The stop test with a loose Lanczos tolerance (1e-8) on the 256^2 x 64
    workload: an L2 pass is confirmed by one more step (Sec. II.C: the Lanczos
    coefficients vanish once the Krylov space is exhausted), so with accurate
    inner solves (1e-11) every frequency stays within 1e-6 (the check sites
    cover all 64, the oracle four of them).  With inner solves at 1e-9 the
    matvec noise keeps some top-level items from ever reaching the test; they
    stop at their step cap, and the report says so (truncated, capped_items)
    instead of returning a silently wrong diagonal."""
    w = synth.SQUARE_256
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 16, 0, PREC_MIXED16, inner_tol=1e-11, lanczos_tol=1e-8, level_streams=3)
    G, rep = p.solve(tV, tom, tsig, report=True)
    print(f"lanczos_tol 1e-8 rep={rep}")
    assert rep["truncated"] == 0
    assert rep["est_rel_err"] < 1e-6
    ks = [0, 1, 21, 63]
    ref = oracle_G(w, V, om, sig, method="rgf", freqs=ks)
    err = oracle.rel_err(G.cpu().numpy()[ks], ref)
    print(f"lanczos_tol 1e-8 oracle err on {ks}: {err:.2e}")
    assert err < 1e-6
    _, rep9 = _plan(w, 16, 0, PREC_MIXED16, inner_tol=1e-9, lanczos_tol=1e-8,
                    level_streams=3).solve(tV, tom, tsig, report=True)
    print(f"inner_tol 1e-9 rep={rep9}")
    assert rep9["est_rel_err"] < 1e-6 or (rep9["truncated"] == 1 and rep9["capped_items"] > 0)


@pytest.mark.parametrize("attempts", [1, 2])
def test_forced_breakdown_restarts(attempts):
    """Host-forced breakdown (the bilinear norm declared vanished at step 3 of
    every open item, Sec. II.A): each affected item is redone from a fresh
    start vector and the result is still exact."""
    w = _case((37, 29), K=3)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    G, rep = _plan(w, 8, 0, 0, fault_step=3, fault_attempts=attempts).solve(tV, tom, tsig,
                                                                             report=True)
    err = oracle.rel_err(G.cpu().numpy(), oracle_G(w, V, om, sig))
    print(f"forced breakdown attempts={attempts} err={err:.2e} rep={rep}")
    assert rep["restarts"] > 0
    assert err < 1e-10


def test_forced_breakdown_exhausts_attempts():
    w = _case((37, 29), K=2)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    with pytest.raises(DysonError) as e:
        _plan(w, 8, 0, 0, fault_step=2, fault_attempts=3).solve(tV, tom, tsig)
    assert e.value.status == 3      # DYSON_EBREAKDOWN


def test_inner_iteration_cap_returns_enoconv():
    w = _case((37, 29), K=2)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    with pytest.raises(DysonError) as e:
        _plan(w, 8, 0, 0, max_inner_iters=1).solve(tV, tom, tsig)
    assert e.value.status == 4      # DYSON_ENOCONV


def test_solve_host_equals_device_solve():
    """dyson_solve_host (host arrays in and out) gives the device result bit
    for bit."""
    w = _case((48, 33), K=3, beta=20.0)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 16, 0, 2)
    Gd = p.solve(tV, tom, tsig).cpu().numpy()
    Gh, rep = p.solve_host(V, om, sig, report=True)
    assert np.array_equal(Gh, Gd)
    assert rep["t_total_ms"] > 0
    with pytest.raises(DysonError) as e:
        bad = om.copy()
        bad[0] = -1.0
        p.solve_host(V, bad, sig)
    assert e.value.status == 1


def test_mixed16_refuses_tiny_imaginary_part():
    """Complex32 factors hold entries up to 1 / min Im H_ii: below 2^-14 the
    complex32 solve is refused up front, blocking and served (instead of
    overflowing FP16 and running every inner solve to its iteration cap)."""
    V, z, sig, mu, tV, tz, tsig = _real_axis((24, 20), K=2, eta=1e-5)
    p16 = Plan((24, 20), t=-1.0, mu=mu, leaf_edge=8, partition=PART_NESTED, precision=2)
    with pytest.raises(DysonError) as e:
        p16.solve_z(tV, tz, tsig)
    assert e.value.status == 6      # DYSON_EUNSUPPORTED
    from paper_1102_3137_amd import MEM_HOST
    with pytest.raises(DysonError) as e:
        p16.submit(V, z, sig, mem=MEM_HOST)
    assert e.value.status == 6


@pytest.mark.parametrize("prec", [1, 2])
def test_solve_cubic_24(prec):
    """24^3 simple cubic lattice (Z = 6, 6^3 tiles, top interface 576 sites) on
    the hardest and easiest Matsubara frequencies at beta = 10, against the
    block-tridiagonal oracle over z-planes."""
    w = synth.Workload(dims=(24, 24, 24), t=-1.0, mu=1.0, vc=1e-3 * (48.0 / 24) ** 2, beta=10.0,
                       freq_index=(0, 31), seed=3, name="cubic 24")
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 6, 0, prec)
    G, rep = p.solve(tV, tom, tsig, report=True)
    ref = oracle_G(w, V, om, sig, method="rgf")
    err = oracle.rel_err(G.cpu().numpy(), ref)
    print(f"24^3 prec={prec} err={err:.2e} rep={rep}")
    assert rep["truncated"] == 0
    assert err < 1e-9


def test_concurrent_levels_match_sequential():
    """The correction levels are independent; running them in concurrent
    groups changes only the order in which the group sums are added."""
    w = _case((96, 80), K=5, beta=20.0)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    G1 = _plan(w, 16, 0, 2, level_streams=1).solve(tV, tom, tsig).cpu().numpy()
    G4 = _plan(w, 16, 0, 2, level_streams=4).solve(tV, tom, tsig).cpu().numpy()
    assert oracle.rel_err(G4, G1) < 1e-13
    assert oracle.rel_err(G4, oracle_G(w, V, om, sig)) < 1e-10


def _dense_periodic(w, V, om, sig, per):
    d = oracle.assemble_diag(V, om, sig, w.mu)
    from oracle import dyson as od
    return np.stack([od.diag_inv_dense(w.dims, d[k], w.t, periodic=per) for k in range(w.n_freq)])


@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "mixed16"])
def test_periodic_uniform_closed_form(prec):
    """Uniform periodic 32x32 lattice, V = Sigma = 0: every G_ii equals
    (1/N) sum_k 1/(i w + mu - eps_k), the plane-wave closed form."""
    w = synth.rect((32, 32), K=3, seed=1, vc=0.0, beta=10.0)
    n, K = w.n_sites, w.n_freq
    om = synth.matsubara(w.beta, w.freq_index)
    dev = torch.device("cuda:0")
    tV = torch.zeros(n, dtype=torch.float64, device=dev)
    tom = torch.from_numpy(om).to(dev)
    tsig = torch.zeros((K, n), dtype=torch.complex128, device=dev)
    p = Plan(w.dims, t=w.t, mu=w.mu, leaf_edge=16, partition=PART_NESTED, precision=prec,
             periodic=(1, 1))
    G = p.solve(tV, tom, tsig).cpu().numpy()
    for k in range(K):
        ref = oracle.closed_form_periodic(w.dims, 1j * om[k] + w.mu, w.t)
        assert np.max(np.abs(G[k] - ref)) / abs(ref) < 1e-10


PERIODIC_CASES = [
    ((48, 32), 8, (1, 0)),       # one wrapped axis, trap and self-energy
    ((24, 32), 8, (1, 1)),       # torus
    ((16, 48), 16, (1, 1)),      # an axis that is one tile wide wraps onto itself
    ((40,), 8, (1,)),            # ring
    ((12, 12, 12), 6, (1, 1, 1)),  # 3-D torus, plane-slice kernels
    ((12, 8, 8), 4, (0, 1, 1)),
    ((4, 8, 8), 4, (1, 0, 0)),   # one tile wide along x: the halo slot wraps onto its own tile
    ((5, 10, 10), 5, (1, 0, 1)),  # the same for the plane-slice kernels
]


@pytest.mark.parametrize("dims,s,per", PERIODIC_CASES, ids=[f"{c[0]}-s{c[1]}-{c[2]}" for c in PERIODIC_CASES])
def test_periodic_solve_vs_dense(dims, s, per):
    w = _case(dims, K=2, mu=1.0 if len(dims) == 3 else 0.5)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = Plan(w.dims, t=w.t, mu=w.mu, leaf_edge=s, partition=PART_NESTED, precision=0,
             periodic=per)
    G, rep = p.solve(tV, tom, tsig, report=True)
    err = oracle.rel_err(G.cpu().numpy(), _dense_periodic(w, V, om, sig, per))
    print(f"{dims} s={s} periodic={per} err={err:.2e} rep={rep}")
    assert rep["truncated"] == 0
    assert err < 1e-10


def _real_axis(dims, K, eta=0.1):
    V, z, sig, mu = synth.real_axis_inputs(dims, K, eta=eta, vc=0.01 * (32.0 / max(dims)) ** 2)
    dev = torch.device("cuda:0")
    return (V, z, sig, mu, torch.from_numpy(V).to(dev), torch.from_numpy(z).to(dev),
            torch.from_numpy(np.ascontiguousarray(sig)).to(dev))


def test_solve_z_on_the_matsubara_axis_is_solve():
    """z_k = i w_k through dyson_solve_z gives bit for bit the dyson_solve result."""
    w = _case((48, 40), K=3)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 8, 0, 2)
    G1 = p.solve(tV, tom, tsig).cpu().numpy()
    tz = (1j * tom.to(torch.complex128)).contiguous()
    G2 = p.solve_z(tV, tz, tsig).cpu().numpy()
    assert np.array_equal(G1, G2)


@pytest.mark.parametrize("iface", [0, 1], ids=["x_form", "interface_form"])
@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "mixed16"])
@pytest.mark.parametrize("dims,s", [((48, 40), 8), ((64, 64), 16), ((10, 9, 8), 4)])
def test_real_axis_vs_oracle(dims, s, prec, iface):
    """Energies w + 0.1i across the band: smaller Im H than on the Matsubara axis."""
    V, z, sig, mu, tV, tz, tsig = _real_axis(dims, K=4)
    p = Plan(dims, t=-1.0, mu=mu, leaf_edge=s, partition=PART_NESTED, precision=prec,
             interface_lanczos=iface)
    G, rep = p.solve_z(tV, tz, tsig, report=True)
    d = oracle.assemble_diag_z(V, z, sig, mu)
    err = oracle.rel_err(G.cpu().numpy(), oracle.oracle_diag(dims, d, -1.0))
    print(f"real axis {dims} s={s} prec={prec} err={err:.2e} rep={rep}")
    assert rep["truncated"] == 0
    assert err < 1e-10


def test_sampled_error_estimate_tracks_accuracy():
    """report.est_rel_err (G_ii against a direct solve of H x = e_i at two
    sites) is at the method's accuracy for a full-rank solve and exposes a
    truncated rank."""
    w = _case((48, 40), K=3)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    G, rep = _plan(w, 8, 0, 2).solve(tV, tom, tsig, report=True)
    err = oracle.rel_err(G.cpu().numpy(), oracle_G(w, V, om, sig))
    assert 0 < rep["est_rel_err"] < 1e-9 and err < 1e-10
    _, rep_t = _plan(w, 8, 0, 2, max_rank=8).solve(tV, tom, tsig, report=True)
    assert rep_t["truncated"] == 1 and rep_t["est_rel_err"] > 1e-4
    _, rep_n = _plan(w, 8, 0, 2, check_sites=0).solve(tV, tom, tsig, report=True)
    assert rep_n["est_rel_err"] == 0.0


SCHUR_CASES = [((32, 32), 16), ((5, 5), 3), ((37, 29), 8), ((48, 33), 16), ((40,), 8),
               ((16, 16), 16), ((9, 8, 7), 4), ((12, 12, 12), 6), ((11, 10, 9), 5)]


@pytest.mark.parametrize("dims,s", SCHUR_CASES, ids=[f"{c[0]}-s{c[1]}" for c in SCHUR_CASES])
def test_explicit_schur_vs_oracle(dims, s):
    """The standard domain-decomposition inverse of Sec. II.B (eq. (6)): S
    formed and inverted explicitly on a one-level decomposition; its diagonal
    equals the oracle's and the low-rank method's."""
    w = _case(dims, K=3, mu=1.0 if len(dims) == 3 else 0.5)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, s, PART_SINGLE, 0)
    G, rep = p.solve_schur(tV, tom, tsig, report=True)
    ref = oracle_G(w, V, om, sig)
    err = oracle.rel_err(G.cpu().numpy(), ref)
    m = p.info.max_m[0] if p.info.levels else 0
    print(f"schur {dims} s={s} m={m} err={err:.2e} rep={rep}")
    assert err < 1e-10
    assert rep["max_rank_used"] == m
    Glr = p.solve(tV, tom, tsig).cpu().numpy()
    assert oracle.rel_err(Glr, ref) < 1e-10


def test_explicit_schur_periodic_and_refusals():
    w = _case((24, 32), K=2)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    per = (1, 1)
    p = Plan(w.dims, t=w.t, mu=w.mu, leaf_edge=8, partition=PART_SINGLE, precision=0,
             periodic=per)
    G = p.solve_schur(tV, tom, tsig).cpu().numpy()
    assert oracle.rel_err(G, _dense_periodic(w, V, om, sig, per)) < 1e-10
    nested = _plan(_case((48, 48), K=1), 8, PART_NESTED, 0)
    assert nested.info.levels > 1
    V1, om1, sig1, tV1, tom1, tsig1 = device_inputs(_case((48, 48), K=1))
    with pytest.raises(DysonError) as e:
        nested.solve_schur(tV1, tom1, tsig1)
    assert e.value.status == 6      # DYSON_EUNSUPPORTED: more than one correction level


def test_cubic_48_stratified_sites():
    """48^3 simple cubic lattice (Z = 6, mu = 1, V = 1e-3 r^2, beta = 10), 6^3
    tiles, nine correction levels (top interface 2304 sites), frequencies w_0
    and w_31, complex32 preconditioner at the library's default tolerances, in
    both forms of the correction, against the exact block-tridiagonal oracle
    (O2) at every site; the error is also reported per stratum of a seeded
    sample: interface sites of every level, leaf sites next to an interface,
    leaf sites away from all of them."""
    import time
    w = synth.Workload(dims=(48, 48, 48), t=-1.0, mu=1.0, vc=1e-3, beta=10.0,
                       freq_index=(0, 31), seed=3, name="cubic 48")
    V, om, sig, tV, tom, tsig = device_inputs(w)
    Gs = []
    for iface in (0, 1):
        pf = _plan(w, 6, PART_NESTED, PREC_MIXED16, interface_lanczos=iface)
        t0 = time.perf_counter()
        G, rep = pf.solve(tV, tom, tsig, report=True)
        Gs.append(G.cpu().numpy())
        print(f"48^3 interface_lanczos={iface}: {time.perf_counter() - t0:.1f} s rep={rep}",
              flush=True)
        assert rep["truncated"] == 0
        p = pf
    depth, is_sep, tile = p.maps()
    n = w.n_sites
    x, y, z = np.arange(n) % 48, (np.arange(n) // 48) % 48, np.arange(n) // 2304
    near = np.zeros(n, bool)
    for dx, dy, dz in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
        xx, yy, zz = x + dx, y + dy, z + dz
        ok = (xx >= 0) & (xx < 48) & (yy >= 0) & (yy < 48) & (zz >= 0) & (zz < 48)
        j = np.where(ok, xx + 48 * (yy + 48 * zz), 0)
        near |= ok & (is_sep[j] == 1)
    rng = np.random.default_rng(17)
    strata = {}
    for lev in range(p.info.levels):
        cand = np.where((is_sep == 1) & (depth == lev))[0]
        strata[f"interface level {lev}"] = rng.choice(cand, min(14, len(cand)), replace=False)
    strata["next to an interface"] = rng.choice(np.where((is_sep == 0) & near)[0], 50, replace=False)
    strata["inside a subdomain"] = rng.choice(np.where((is_sep == 0) & ~near)[0], 50, replace=False)
    assert sum(len(v) for v in strata.values()) >= 200
    d = oracle.assemble_diag(V, om, sig, w.mu)
    err = {"X": 0.0, "interface": 0.0}
    for k in range(2):
        t0 = time.perf_counter()
        ref = oracle.diag_inv_rgf(w.dims, d[k], w.t)
        for form, G in zip(("X", "interface"), Gs):
            e = np.abs(G[k] - ref) / np.abs(ref)
            err[form] = max(err[form], float(e.max()))
            worst = {name: float(e[s_].max()) for name, s_ in strata.items()}
            print(f"48^3 w_{w.freq_index[k]} ({form} form): oracle {time.perf_counter() - t0:.0f} s, "
                  f"max over every site {e.max():.2e}; per stratum {worst}", flush=True)
    # the interface form's top level inverts a 2304 x 2304 projected Hessenberg
    # matrix: its diag(S^-1) on those interface sites lands at 1.4e-10..1.9e-10
    # at w_0 (every other site and w_31 below 1e-10)
    assert err["X"] < 1e-10 and err["interface"] < 3e-10


@pytest.mark.parametrize("dims,s,part,iface", [((48, 33), 8, 0, 0), ((48, 33), 8, 0, 1),
                                               ((12, 12, 12), 6, 0, 0), ((9, 8, 7), 4, 1, 1)])
def test_inner_graphs_match_direct_launches(dims, s, part, iface):
    """The inner solves' iteration chunks replayed as captured HIP graphs give
    the results of direct launches bit for bit, on every replay: two graph
    solves around a direct one, and a repeat after a solve with other
    inputs."""
    w = _case(dims, K=3, mu=1.0 if len(dims) == 3 else 0.5)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    pg = _plan(w, s, part, 0, interface_lanczos=iface)
    pd = _plan(w, s, part, 0, interface_lanczos=iface, inner_graphs=-1)
    G1 = pg.solve(tV, tom, tsig).cpu().numpy()
    Gd = pd.solve(tV, tom, tsig).cpu().numpy()
    G2 = pg.solve(tV, tom, tsig).cpu().numpy()
    assert np.array_equal(G1, Gd) and np.array_equal(G2, Gd)
    pg.solve(tV * 0.5, tom, tsig)          # other inputs through the same graphs
    assert np.array_equal(pg.solve(tV, tom, tsig).cpu().numpy(), Gd)
    assert oracle.rel_err(Gd, oracle_G(w, V, om, sig)) < 1e-10
