"""GPU parity of the flexible conjugate gradient (FCG / GCC / IPCG) with refreshed sketches: the HIP
library through its C ABI against the CPU oracle on the same draws, iterate by iterate through the
exact-error trace, plus edge cases and properties that hold at any size.

Tolerances: every sketch is FP64 on both sides (the Gaussian normals within a few ulp of the
oracle's), so iterates agree to the rounding of the factorizations and passes (relative A-norm
difference 1e-10 of ||A x*||)."""
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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = [
    # kind, n, d, m, window, refresh, iters
    ("srht", 4096, 32, 128, 1, 1, 8),
    ("srht", 4096, 32, 128, 100, 1, 8),
    ("srht", 3000, 37, 150, 0, 1, 6),
    ("sjlt", 4096, 32, 128, 2, 1, 8),
    ("sjlt", 2500, 21, 90, 100, 1, 10),
    ("gaussian", 4096, 32, 128, 1, 1, 6),
    ("srht", 4096, 32, 128, 3, 0, 8),
]


@pytest.mark.parametrize("kind,n,d,m,window,refresh,T", CASES)
def test_fcg_iterates(ctx, kind, n, d, m, window, refresh, T):
    import torch

    from oracle.fcg import fcg
    from oracle.solve import lstsq_householder
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    say("fcg", kind, n, d, m, window, refresh, T)
    P = make_problem(n, d, 1e4, sigma=0.01, seed=16)
    A, y = P["A"], P["y"]
    s = 2 if kind == "sjlt" else 1
    xs = lstsq_householder(A, y)
    its = fcg(A, y, kind, m, seed=91, k=window, iters=T, refresh=bool(refresh), s=s)
    x = torch.zeros(d, dtype=torch.float64, device="cuda")
    trace = torch.zeros(T + 1, dtype=torch.float64, device="cuda")
    info = ctx.fcg_solve(dev(A), dev(y), lsq.sketch_desc(kind, m, seed=91, s=s), x, iters=T, window=window,
                         refresh=refresh, x_ref=dev(xs), err_trace=trace)
    assert info.iters == T
    scale = np.linalg.norm(A @ xs)
    diff = np.linalg.norm(A @ (host(x) - its[-1])) / scale
    tol = 1e-10
    e_or = np.array([np.linalg.norm(A @ (xt - xs)) / scale for xt in its])
    e_gpu = host(trace)
    say("  diff", diff, "final error", e_or[-1], "gpu", e_gpu[-1])
    assert diff <= tol
    # the exact-error trace: each entry within the same tolerance of the oracle's
    assert np.all(np.abs(e_gpu - e_or) <= tol + 1e-9 * e_or)
    # exact line searches never increase the A-norm error
    assert np.all(np.diff(e_gpu) <= 1e-12)


def test_fcg_fixed_sketch_matches_pcg(ctx):
    """With refresh = 0, FCG with any window k >= 1 is PCG (the library's own PCG, same sketch)."""
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_problem
    n, d, m, T = 8192, 48, 192, 12
    P = make_problem(n, d, 1e5, sigma=0.01, seed=17)
    A, y = dev(P["A"]), dev(P["y"])
    desc = lsq.sketch_desc("srht", m, seed=5)
    x_pcg = torch.zeros(d, dtype=torch.float64, device="cuda")
    st, _ = ctx.pcg_solve(A, y, desc, x_pcg, tol=1e-30, max_iter=T, raise_on_error=False)
    assert st == lsq.LSQ_ERR_NOT_CONVERGED
    An = P["A"]
    scale = np.linalg.norm(An @ np.linalg.lstsq(An, P["y"], rcond=None)[0])
    for k in (1, 4, T):
        x = torch.zeros(d, dtype=torch.float64, device="cuda")
        ctx.fcg_solve(A, y, desc, x, iters=T, window=k, refresh=0)
        diff = np.linalg.norm(An @ (host(x) - host(x_pcg))) / scale
        say("  fixed sketch k", k, "diff vs PCG", diff)
        assert diff <= 1e-9


def test_gcc_terminates_in_d_steps(ctx):
    import torch

    from oracle.solve import lstsq_householder
    from paper_1911_02675_amd import lsq
    from synth import make_problem
    n, d, m = 2048, 6, 24
    P = make_problem(n, d, 1e3, sigma=0.01, seed=18)
    A, y = P["A"], P["y"]
    xs = lstsq_householder(A, y)
    for kind in ("srht", "sjlt", "gaussian"):
        x = torch.zeros(d, dtype=torch.float64, device="cuda")
        tr = torch.zeros(d + 1, dtype=torch.float64, device="cuda")
        ctx.fcg_solve(dev(A), dev(y), lsq.sketch_desc(kind, m, seed=3, s=2), x, iters=d, window=d,
                      x_ref=dev(xs), err_trace=tr)
        e = host(tr)
        say("  GCC", kind, "error after d steps", e[-1])
        assert e[-1] <= 1e-9


def test_fcg_edge_cases(ctx):
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_problem
    P = make_problem(1024, 16, 1e2, sigma=0.01, seed=19)
    A, y = dev(P["A"]), dev(P["y"])
    desc = lsq.sketch_desc("srht", 64, seed=2)
    x = torch.full((16,), 0.5, dtype=torch.float64, device="cuda")
    info = ctx.fcg_solve(A, y, desc, x, iters=0, window=1)  # no iterations: x unchanged
    assert info.iters == 0 and np.all(host(x) == 0.5)
    with pytest.raises(lsq.LsqError) as e:
        ctx.fcg_solve(A, y, desc, x, iters=4, window=-1)
    assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
    tr = torch.zeros(5, dtype=torch.float64, device="cuda")
    with pytest.raises(lsq.LsqError) as e:
        ctx.fcg_solve(A, y, desc, x, iters=4, window=1, err_trace=tr)  # trace without x_ref
    assert e.value.status == lsq.LSQ_ERR_INVALID_ARG
    with pytest.raises(lsq.LsqError) as e:
        ctx.fcg_solve(A, y, desc, x, iters=2000, window=1500)
    assert e.value.status == lsq.LSQ_ERR_UNSUPPORTED
    assert np.all(host(x) == 0.5)  # argument errors leave x untouched
    # a window larger than the number of iterations is GCC; an exact solution is a fixed point
    xs = torch.from_numpy(np.linalg.lstsq(P["A"], P["y"], rcond=None)[0]).cuda()
    x2 = xs.clone()
    ctx.fcg_solve(A, y, desc, x2, iters=3, window=50)
    assert float(torch.linalg.norm(A @ (x2 - xs))) <= 1e-12 * float(torch.linalg.norm(A @ xs))
