"""GPU tests of the interface form of the correction (opts.interface_lanczos):
bilinear Lanczos on the Schur complement S of each correction domain for
exactly m steps, the projected Hessenberg matrix inverted per (domain,
frequency), diag(X) = diag(V H^{-1} V^T).  Against the CPU oracle at the same
tolerances as the X form (1e-10 in FP64 at full interface rank)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import device_inputs, oracle_G, have_gpu

pytestmark = pytest.mark.gpu

if have_gpu():
    import torch
    from paper_1102_3137_amd import Plan, PART_NESTED, PART_SINGLE, PREC_MIXED16, DysonError


def _case(dims, K=2, seed=7, vc=None, beta=10.0, mu=0.5):
    if vc is None:
        vc = 0.01 * (32.0 / max(dims)) ** 2
    return synth.rect(dims, K=K, seed=seed, vc=vc, mu=mu, beta=beta)


def _plan(w, s, part=0, prec=0, **kw):
    return Plan(w.dims, t=w.t, mu=w.mu, leaf_edge=s, partition=part, precision=prec,
                interface_lanczos=1, **kw)


IFACE_CASES = [
    (synth.SMALL_32, 16, 1),                     # one level, m = 63
    (synth.SMALL_32, 16, 0),                     # recursive bisection
    (_case((37, 29), K=3), 8, 0),                # ragged tiles, several levels
    (_case((5, 5), K=2), 3, 1),                  # m = 9
    (_case((40,), K=2), 8, 0),                   # chain: m = 1 per domain
    (_case((16, 16), K=2), 16, 0),               # a single leaf: no correction level
    (_case((48, 33), K=4, beta=20.0), 16, 0),    # uneven halves
    (_case((9, 8, 7), K=2, mu=1.0), 4, 0),       # cubic, ragged tiles
    (_case((12, 12, 12), K=3, mu=1.0), 6, 0),    # cubic, plane-slice inner kernels
    (_case((13, 11, 10), K=2, mu=1.0), 5, 1),    # cubic, one level
]


@pytest.mark.parametrize("w,s,part", IFACE_CASES, ids=[f"{c[0].dims}-s{c[1]}-p{c[2]}" for c in IFACE_CASES])
@pytest.mark.parametrize("prec", [0, 2], ids=["fp64", "mixed16"])
def test_interface_form_vs_oracle(w, s, part, prec):
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, s, part, prec)
    G, rep = p.solve(tV, tom, tsig, report=True)
    ref = oracle_G(w, V, om, sig)
    err = oracle.rel_err(G.cpu().numpy(), ref)
    print(f"iface {w.dims} s={s} part={part} prec={prec} err={err:.2e} rep={rep}", flush=True)
    assert err < 1e-10
    assert rep["truncated"] == 0
    # exactly m steps per domain: the largest rank used is the largest interface
    if p.info.levels:
        assert rep["max_rank_used"] == max(p.info.max_m[:p.info.levels])


@pytest.mark.parametrize("dims,s,part", [((32, 32), 16, 1), ((37, 29), 8, 0), ((9, 8, 7), 4, 0)])
def test_interface_level_equals_dense_diag_X(dims, s, part):
    """One level in the interface form adds diag(X) of every domain of the
    level (X = H_D^{-1} - blkdiag(B_D^{-1}, 0), dense) after exactly m steps."""
    from tests.test_gpu_parity import _dense_X_diag
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
        m, cap = p.domains(level)
        assert np.array_equal(steps, np.broadcast_to(m[None, :], steps.shape)), (level, steps, m)


def _uniform_inputs(w):
    n, K = w.n_sites, w.n_freq
    om = synth.matsubara(w.beta, w.freq_index)
    dev = torch.device("cuda:0")
    return (np.zeros(n), om, np.zeros((K, n), complex),
            torch.zeros(n, dtype=torch.float64, device=dev), torch.from_numpy(om).to(dev),
            torch.zeros((K, n), dtype=torch.complex128, device=dev))


def test_uniform_square_with_repeated_eigenvalues():
    """V = Sigma = 0 on an open 31x31 lattice split by a centred cross: the
    four 15x15 quadrants are congruent, and S has 15 doubled eigenvalues, so
    in exact arithmetic a Krylov space of S stops short of the interface.
    Rounding supplies the missing directions (the residual never reaches the
    noise level) and the result is exact."""
    w = synth.rect((31, 31), K=2, seed=1, vc=0.0, beta=10.0)
    V, om, sig, tV, tom, tsig = _uniform_inputs(w)
    p = _plan(w, 16, PART_SINGLE)
    G, rep = p.solve(tV, tom, tsig, report=True)
    err = oracle.rel_err(G.cpu().numpy(), oracle_G(w, V, om, sig, method="dense"))
    print(f"uniform 31^2 err={err:.2e} rep={rep}", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("part", [1, 0])
def test_invariant_subspace_continuation(part):
    """t = 0 with a uniform potential: S = d I on every interface, so each
    step's residual vanishes and the basis continues from a fresh random
    real direction (a zero below the diagonal of H) every step; after m steps
    it spans the interface and G = 1/d.  (A Krylov space of X itself
    has dimension one here.)"""
    w = synth.Workload(dims=(32, 32), t=0.0, mu=0.5, vc=0.0, beta=10.0, freq_index=(0, 5),
                       seed=1, name="decoupled 32")
    V, om, sig, tV, tom, tsig = _uniform_inputs(w)
    p = _plan(w, 16, part)
    G, rep = p.solve(tV, tom, tsig, report=True)
    ref = oracle_G(w, V, om, sig, method="dense")
    err = oracle.rel_err(G.cpu().numpy(), ref)
    fresh = sum(int(np.sum(p.domains(l)[0] - 1)) for l in range(p.info.levels)) * w.n_freq
    print(f"t=0 part={part} err={err:.2e} rep={rep} continuations>={fresh}", flush=True)
    assert err < 1e-10
    assert rep["restarts"] >= fresh


def test_periodic_uniform_closed_form_interface():
    w = synth.rect((32, 32), K=3, seed=1, vc=0.0, beta=10.0)
    n, K = w.n_sites, w.n_freq
    om = synth.matsubara(w.beta, w.freq_index)
    dev = torch.device("cuda:0")
    tV = torch.zeros(n, dtype=torch.float64, device=dev)
    tom = torch.from_numpy(om).to(dev)
    tsig = torch.zeros((K, n), dtype=torch.complex128, device=dev)
    p = Plan(w.dims, t=w.t, mu=w.mu, leaf_edge=16, partition=PART_NESTED, precision=0,
             periodic=(1, 1), interface_lanczos=1)
    G = p.solve(tV, tom, tsig).cpu().numpy()
    for k in range(K):
        ref = oracle.closed_form_periodic(w.dims, 1j * om[k] + w.mu, w.t)
        assert np.max(np.abs(G[k] - ref)) / abs(ref) < 1e-10


@pytest.mark.parametrize("L,freqs,prec", [(128, (0, 63), 0), (256, (0, 31, 63), 0)])
def test_interface_form_large_lattice(L, freqs, prec):
    w = synth.Workload(dims=(L, L), t=-1.0, mu=0.5, vc=2e-4 * (256.0 / L) ** 2, beta=20.0,
                       freq_index=tuple(freqs), seed=2, name=f"square {L}")
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 16, 0, prec)
    G, rep = p.solve(tV, tom, tsig, report=True)
    err = oracle.rel_err(G.cpu().numpy(), oracle_G(w, V, om, sig, method="rgf"))
    print(f"iface {L}^2 freqs={freqs} prec={prec} err={err:.2e} rep={rep}", flush=True)
    assert rep["truncated"] == 0
    assert err < 1e-10


def test_interface_form_bench_configuration_256():
    """The throughput workload's settings (complex32 factors, inner solves to
    1e-11, six concurrent level groups) in the interface form."""
    w = synth.Workload(dims=(256, 256), t=-1.0, mu=0.5, vc=2e-4, beta=20.0,
                       freq_index=(0, 31, 63), seed=2, name="square 256")
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 16, 0, PREC_MIXED16, inner_tol=1e-11, lanczos_tol=1e-11, level_streams=6)
    G, rep = p.solve(tV, tom, tsig, report=True)
    err = oracle.rel_err(G.cpu().numpy(), oracle_G(w, V, om, sig, method="rgf"))
    print(f"iface bench configuration err={err:.2e} rep={rep}", flush=True)
    assert rep["truncated"] == 0
    assert err < 1e-8


def test_interface_form_forced_breakdown_restarts():
    """Host-forced breakdown at step 3 of every open item: the items are
    redone from fresh start vectors (Hessenberg columns cleared) and the
    result is exact; forced on every attempt the call fails."""
    w = _case((37, 29), K=3)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    G, rep = _plan(w, 8, 0, fault_step=3, fault_attempts=2).solve(tV, tom, tsig, report=True)
    err = oracle.rel_err(G.cpu().numpy(), oracle_G(w, V, om, sig))
    print(f"iface forced breakdown err={err:.2e} rep={rep}", flush=True)
    assert rep["restarts"] > 0
    assert err < 1e-10
    with pytest.raises(DysonError) as e:
        _plan(w, 8, 0, fault_step=2, fault_attempts=3).solve(tV, tom, tsig)
    assert e.value.status == 3      # DYSON_EBREAKDOWN


def test_interface_form_matches_x_form_and_is_deterministic():
    w = _case((48, 33), K=3, beta=20.0)
    V, om, sig, tV, tom, tsig = device_inputs(w)
    p = _plan(w, 8, 0)
    G1 = p.solve(tV, tom, tsig).cpu().numpy()
    G2 = p.solve(tV, tom, tsig).cpu().numpy()
    assert np.array_equal(G1, G2)
    Gk = p.solve(tV, tom[1:2].contiguous(), tsig[1:2].contiguous()).cpu().numpy()
    assert np.array_equal(Gk[0], G1[1])
    px = Plan(w.dims, t=w.t, mu=w.mu, leaf_edge=8, partition=0, precision=0)
    Gx = px.solve(tV, tom, tsig).cpu().numpy()
    assert oracle.rel_err(G1, Gx) < 2e-10


def test_interface_form_refuses_rank_cap():
    w = synth.SMALL_32
    with pytest.raises(DysonError) as e:
        _plan(w, 16, 1, max_rank=32)
    assert e.value.status == 1
