"""The allocation-free entry point (dyson_solve_noalloc) called through the C
ABI: its result equals dyson_solve's with the levels in sequence, on two calls
in a row (the second with a smaller input), it allocates no device memory,
and a workspace beyond the scratch array is refused up front."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import device_inputs, oracle_G, have_gpu

pytestmark = pytest.mark.gpu

if have_gpu():
    import torch
    from paper_1102_3137_amd import Plan, DysonError, PREC_MIXED16, PREC_FP64
    from paper_1102_3137_amd import binding as B


def _case(dims, K, seed=5):
    return synth.rect(dims, K=K, seed=seed, vc=0.01 * (32.0 / max(dims)) ** 2, beta=20.0)


@pytest.mark.parametrize("iface", [0, 1], ids=["x_form", "interface_form"])
def test_noalloc_matches_solve_twice_then_smaller(iface):
    w1 = _case((48, 33), K=4)
    w2 = _case((32, 32), K=2, seed=6)
    cases = []
    for w, prec in ((w1, PREC_MIXED16), (w2, PREC_FP64)):
        V, om, sig, tV, tom, tsig = device_inputs(w)
        p = Plan(w.dims, t=w.t, mu=w.mu, leaf_edge=16, precision=prec, level_streams=1,
                 interface_lanczos=iface)
        assert 0 < p.noalloc_bytes(w.n_freq) <= B.dyson_noalloc_max_bytes()
        ref = p.solve(tV, tom, tsig)               # the allocating path, levels in sequence
        G = torch.empty_like(ref)
        cases.append((w, p, V, om, sig, tV, tom, tsig, ref, G))
    w, p, V, om, sig, tV, tom, tsig, ref, _ = cases[0]
    G3 = torch.full((2, w.n_sites), complex(float("nan"), float("nan")), dtype=torch.complex128,
                    device="cuda:0")
    tom2, tsig2 = tom[:2].contiguous(), tsig[:2].contiguous()
    for c in cases:
        c[9].fill_(complex(float("nan"), float("nan")))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    # first call on the larger input, then the smaller plan, then the larger
    # plan again with fewer frequencies; every buffer above is the caller's
    reps = []
    for w, p, V, om, sig, tV, tom, tsig, ref, G in cases:
        _, rep = p.solve_noalloc(tV, tom, tsig, G, report=True)
        reps.append(rep)
    cases[0][1].solve_noalloc(cases[0][5], tom2, tsig2, G3)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    outs = [(c[9], r) for c, r in zip(cases, reps)]
    # no device allocation by the library (a little slack for runtime bookkeeping)
    assert free0 - free1 < (8 << 20), (free0, free1)
    for (Gn, rep), (w, p, V, om, sig, tV, tom, tsig, ref, _) in zip(outs, cases):
        assert torch.equal(Gn, ref)
        assert rep["truncated"] == 0 and rep["hbm_bytes"] == p.noalloc_bytes(w.n_freq)
        err = oracle.rel_err(Gn.cpu().numpy(), oracle_G(w, V, om, sig))
        assert err < 1e-10, err
    assert torch.equal(G3, cases[0][8][:2])


def test_noalloc_refuses_beyond_scratch():
    w = synth.Workload(dims=(256, 256), t=-1.0, mu=0.5, vc=2e-4, beta=20.0,
                       freq_index=tuple(range(64)), seed=2, name="square 256")
    p = Plan(w.dims, t=w.t, mu=w.mu, leaf_edge=16, precision=PREC_MIXED16, level_streams=1)
    assert p.noalloc_bytes(64) > B.dyson_noalloc_max_bytes()
    n = w.n_sites
    tV = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    tom = torch.ones(64, dtype=torch.float64, device="cuda:0")
    tsig = torch.zeros((64, n), dtype=torch.complex128, device="cuda:0")
    G = torch.empty((64, n), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(DysonError) as e:
        p.solve_noalloc(tV, tom, tsig, G)
    assert e.value.status == 1 and "maximum" in str(e.value)
