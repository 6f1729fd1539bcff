"""GPU parity of fixed-sketch IHS / Polyak-IHS with the Theorem 3.2 parameters (rho = d/m,
lsq_ihs_opts.mu_rule 2 and 3) against the CPU oracle on the same draws.  Tolerances as for the other
IHS parity tests: every sketch is FP64 on both sides (the Gaussian normals within a few ulp), so the
iterates agree to rounding (1e-10 of ||A x*||)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1911_02675_amd import lsq
    c = lsq.Context()
    yield c
    c.close()


@pytest.mark.parametrize("kind,rule", [("srht", 2), ("srht", 3), ("sjlt", 3), ("gaussian", 2)])
def test_fixed_sketch_rules(ctx, kind, rule):
    import torch

    from oracle import theory
    from oracle.ihs import ihs
    from oracle.solve import lstsq_householder
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    say("fixed-sketch rule", kind, rule)
    n, d, m, T = 4096, 32, 128, 10
    P = make_problem(n, d, 1e4, sigma=0.01, seed=8)
    A, y = P["A"], P["y"]
    s = 2 if kind == "sjlt" else 1
    mu_i, _, mu_p, beta_p = theory.fixed_sketch_params(d, m)
    mu, beta = (mu_i, 0.0) if rule == 2 else (mu_p, beta_p)
    its = ihs(A, y, kind, m, seed=55, mu=mu, beta=beta, iters=T, refresh=False, s=s)
    x = torch.zeros(d, dtype=torch.float64, device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    info = ctx.ihs_solve(dev(A), dev(y), lsq.sketch_desc(kind, m, seed=55, s=s), x, iters=T,
                         beta=0.0 if rule == 2 else 0.3, refresh=0, mu_rule=rule)
    assert abs(info.mu - mu) <= 1e-14
    xs = lstsq_householder(A, y)
    torch.cuda.synchronize()
    diff = np.linalg.norm(A @ (x.cpu().numpy() - its[-1])) / np.linalg.norm(A @ xs)
    say("  diff", diff)
    assert diff <= 1e-10


def test_fixed_sketch_rule_needs_m_above_d(ctx):
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_problem
    P = make_problem(256, 16, 1e2, sigma=0.01, seed=9)
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    with pytest.raises(lsq.LsqError) as e:
        ctx.ihs_solve(dev(P["A"]), dev(P["y"]), lsq.sketch_desc("sjlt", 16, seed=1, s=2), x, iters=2,
                      refresh=0, mu_rule=2)
    assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
    with pytest.raises(lsq.LsqError) as e:
        ctx.ihs_solve(dev(P["A"]), dev(P["y"]), lsq.sketch_desc("sjlt", 64, seed=1, s=2), x, iters=2,
                      refresh=0, mu_rule=4)
    assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
