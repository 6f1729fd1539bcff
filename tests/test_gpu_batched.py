"""GPU parity of the batched form (lsq_pcg_solve_batched, one persistent launch for many problems)
against the CPU oracle, through the C ABI.

Per problem: the returned R (Householder factor of the SJLT sketch S A, diag > 0) against the
oracle's R of the oracle's S A with the same draws, to O(eps kappa); the solution against the
oracle's direct solve in the relative A-norm (1e-10, or four times the disagreement of two
backward-stable FP64 solvers where conditioning limits every solver).  The batch mixes FP32 and
FP64 storage, aligned, padded (padding filled with NaN) and misaligned layouts, every column
mapping of the kernel, d from 1 to 256 and m from d to 1024."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _torch():
    import torch
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1911_02675_amd import lsq
    c = lsq.Context()
    yield c
    c.close()


def host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


class Case:
    """One problem: stored matrix (with its layout on the device), y, sketch parameters."""

    def __init__(self, n, d, m, s, dtype, kappa, layout="contig", lda=None, seed=0, dup_col=False):
        from synth import make_problem
        torch = _torch()
        P = make_problem(n, d, kappa, sigma=0.01, seed=1000 + seed)
        A = P["A"]
        if dup_col:
            A[:, d - 1] = A[:, 0]
        self.A_host = A.astype(np.float32) if dtype == "f32" else A
        self.A64 = self.A_host.astype(np.float64)
        self.y = P["y"]
        self.n, self.d, self.m, self.s, self.kappa = n, d, m, s, kappa
        self.seed, self.t = 500 + seed, seed % 3
        tdt = torch.float32 if dtype == "f32" else torch.float64
        lda = lda or d
        if layout == "misaligned":
            buf = torch.full((n * lda + 1,), float("nan"), dtype=tdt, device="cuda")
            self.A_dev = buf[1:].view(n, lda)[:, :d]
        else:
            buf = torch.full((n, lda), float("nan"), dtype=tdt, device="cuda")
            self.A_dev = buf[:, :d]
        self.A_dev.copy_(torch.from_numpy(self.A_host).cuda())
        self._keep = buf
        self.y_dev = torch.from_numpy(self.y).cuda()
        self.x = torch.zeros(d, dtype=torch.float64, device="cuda")
        self.R = torch.zeros((d, d), dtype=torch.float64, device="cuda")

    def desc(self):
        from paper_1911_02675_amd import lsq
        return lsq.sketch_desc("sjlt", self.m, seed=self.seed, t=self.t, s=self.s)

    def oracle_r(self):
        from oracle.householder import householder_qr
        from oracle.sketch import sjlt_sketch
        return householder_qr(sjlt_sketch(self.A64, self.m, self.s, self.seed, self.t))

    def oracle_x(self):
        from oracle.solve import a_norm_error, lstsq_householder
        x1 = lstsq_householder(self.A64, self.y, block_rows=8192)
        x2 = np.linalg.lstsq(self.A64, self.y, rcond=None)[0]
        return x1, a_norm_error(self.A64, x2, x1)


# (n, d, m, s, dtype, kappa, layout, lda): every column mapping of the kernel appears at least once
CASES = [
    (4096, 16, 64, 4, "f32", 1e3, "contig", None),       # FP32, 4 lanes per row
    (3000, 17, 68, 4, "f32", 1e4, "contig", None),       # lda 17: element loads
    (3001, 17, 68, 4, "f32", 1e4, "padded", 20),         # 16-byte rows, straddling chunk, NaN padding
    (20000, 256, 1024, 4, "f32", 1e6, "contig", None),   # 64 lanes per row, largest m
    (5000, 100, 400, 2, "f64", 1e5, "contig", None),     # FP64, 64 lanes, one chunk
    (6000, 200, 800, 8, "f64", 1e2, "contig", None),     # FP64, two chunks per lane
    (2500, 5, 20, 1, "f64", 10.0, "contig", None),       # FP64, 8 lanes, s = 1
    (1000, 1, 4, 3, "f64", 1.0, "contig", None),         # d = 1
    (256, 256, 1024, 4, "f32", 1e3, "contig", None),     # square
    (4099, 33, 33, 4, "f32", 1e2, "padded", 36),         # m = d
    (7000, 130, 520, 4, "f64", 1e4, "padded", 131),      # odd lda: element loads, FP64
    (4500, 64, 256, 4, "f32", 1e3, "misaligned", None),  # A not 16-byte aligned
    (3333, 48, 200, 16, "f32", 1e5, "contig", None),     # s = 16
    (12000, 150, 600, 4, "f32", 1e6, "padded", 152),     # 64 lanes, ragged d
]


def _make(cases):
    return [Case(n, d, m, s, dt, k, layout=lay, lda=lda, seed=i)
            for i, (n, d, m, s, dt, k, lay, lda) in enumerate(cases)]


def _run(ctx, cs, raise_on_error=True):
    return ctx.pcg_solve_batched([c.A_dev for c in cs], [c.y_dev for c in cs], [c.desc() for c in cs],
                                 [c.x for c in cs], tol=1e-10, max_iter=300, mixed=1, max_refine=10,
                                 Rs=[c.R for c in cs], raise_on_error=raise_on_error)


def _check_case(c, info):
    from oracle.solve import a_norm_error
    Rg = host(c.R)
    Ro = c.oracle_r()
    assert np.all(np.diag(Rg) > 0) and np.allclose(np.tril(Rg, -1), 0)
    kap_sa = np.linalg.cond(Ro)
    dr = np.abs(Rg - Ro).max() / np.abs(Ro).max()
    xs, fl = c.oracle_x()
    e = a_norm_error(c.A64, host(c.x), xs)
    # The stop rule 4 sqrt(rho_t / rho_0) <= tol bounds e_A only up to the conditioning of the
    # preconditioned matrix: e_A(t) / e_A(0) <= kappa(A R^{-1}) sqrt(rho_t / rho_0), so the
    # guaranteed level is tol kappa(A R^{-1}) / 4 (about tol for m >= 4d, larger as m -> d).
    kap_pre = np.linalg.cond(c.A64 @ np.linalg.inv(Ro))
    say(f"  n={c.n} d={c.d} m={c.m} s={c.s} kappa={c.kappa:g}: R rel diff {dr:.2e} "
        f"(cond {kap_sa:.1e}), e_A {e:.2e} (floor {fl:.1e}, cond(A R^-1) {kap_pre:.1f}), "
        f"iters {info.iters} refinements {info.refinements} est {info.est_rel_err:.1e}")
    assert dr <= 50 * c.m * EPS * kap_sa
    assert info.status == 0
    assert e <= max(1e-10, 4 * fl) * max(1.0, kap_pre / 4)


def test_batched_mixed_shapes(ctx):
    say("batched: 14 problems")
    cs = _make(CASES)
    st, infos = _run(ctx, cs)
    assert st == 0
    for c, info in zip(cs, infos):
        _check_case(c, info)


def test_batched_matches_single_problem_solver(ctx):
    """Same draws, same algorithm: the batched solution and the single-problem solver's agree."""
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    torch = _torch()
    cs = _make(CASES[:5])
    st, infos = _run(ctx, cs)
    for c, info in zip(cs, infos):
        x1 = torch.zeros(c.d, dtype=torch.float64, device="cuda")
        st1, inf1 = ctx.pcg_solve(c.A_dev, c.y_dev, c.desc(), x1, tol=1e-10, mixed=1, max_refine=10,
                                  max_iter=300)
        diff = a_norm_error(c.A64, host(c.x), host(x1))
        say(f"  d={c.d}: batched iters {info.iters}, single {inf1.iters}, e_A diff {diff:.1e}")
        assert diff <= 3e-10
        assert abs(info.iters - inf1.iters) <= max(3, inf1.iters // 10)


def test_batched_slots_do_not_change_results(ctx):
    """A problem's arithmetic does not depend on which workgroup takes it: solutions are bitwise
    equal for 1, 3 and the default number of workgroups (queue recycling)."""
    from paper_1911_02675_amd import lsq
    cases = CASES[:4] + CASES[6:9]
    ref = None
    for slots in (0, 3, 1):
        lsq.tune("batched_slots", slots)
        try:
            cs = _make(cases)
            st, infos = _run(ctx, cs)
        finally:
            lsq.tune("batched_slots", 0)
        xs = [host(c.x) for c in cs]
        say(f"  slots {slots}: iters {[i.iters for i in infos]}")
        if ref is None:
            ref = xs
        else:
            for a, b in zip(ref, xs):
                assert np.array_equal(a, b)


def test_batched_graph_replay(ctx):
    """The second call with the same batch shape replays the captured graph; new data each time,
    every replay checked against the oracle, with eager work and synchronisation in between."""
    from oracle.solve import a_norm_error
    torch = _torch()
    cases = [CASES[0], CASES[4], CASES[6]]
    for rep in range(3):
        cs = [Case(n, d, m, s, dt, k, layout=lay, lda=lda, seed=10 * rep + i)
              for i, (n, d, m, s, dt, k, lay, lda) in enumerate(cases)]
        st, infos = _run(ctx, cs)
        torch.cuda.synchronize()
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()  # eager work between replays
        for c, info in zip(cs, infos):
            xs, fl = c.oracle_x()
            e = a_norm_error(c.A64, host(c.x), xs)
            say(f"  replay {rep} d={c.d}: e_A {e:.1e}")
            assert info.status == 0 and e <= max(1e-10, 4 * fl)


def test_batched_single_and_plain_pcg(ctx):
    """count = 1, and the plain (non-refined) PCG of the batched kernel."""
    from oracle.solve import a_norm_error
    cs = _make([CASES[4]])
    st, infos = ctx.pcg_solve_batched([cs[0].A_dev], [cs[0].y_dev], [cs[0].desc()], [cs[0].x],
                                      tol=1e-10, max_iter=300, mixed=0)
    xs, fl = cs[0].oracle_x()
    e = a_norm_error(cs[0].A64, host(cs[0].x), xs)
    say(f"  plain PCG: e_A {e:.1e}, iters {infos[0].iters}")
    assert st == 0 and infos[0].refinements == 0 and e <= max(1e-10, 4 * fl)


def test_batched_rank_deficient_problem_reported(ctx):
    """A problem whose S A is rank deficient gets LSQ_ERR_RANK; the others are solved."""
    from paper_1911_02675_amd import lsq
    cs = _make(CASES[:2])
    cs.append(Case(2000, 12, 48, 4, "f64", 10.0, seed=77, dup_col=True))
    st, infos = _run(ctx, cs, raise_on_error=False)
    say("  statuses", [i.status for i in infos])
    assert st == lsq.LSQ_ERR_RANK
    assert infos[2].status == lsq.LSQ_ERR_RANK
    assert infos[0].status == 0 and infos[1].status == 0
    for c, info in zip(cs[:2], infos[:2]):
        _check_case(c, info)


def test_batched_argument_errors(ctx):
    from paper_1911_02675_amd import lsq
    torch = _torch()
    c = _make([CASES[0]])[0]

    def call(desc=None, A=None, x=None):
        return ctx.pcg_solve_batched([c.A_dev if A is None else A], [c.y_dev], [desc or c.desc()],
                                     [c.x if x is None else x], raise_on_error=False)[0]

    assert call(desc=lsq.sketch_desc("srht", 64, seed=1)) == lsq.LSQ_ERR_UNSUPPORTED
    assert call(desc=lsq.sketch_desc("sjlt", 2048, seed=1, s=4)) == lsq.LSQ_ERR_UNSUPPORTED
    assert call(desc=lsq.sketch_desc("sjlt", 8, seed=1, s=4)) == lsq.LSQ_ERR_UNSUPPORTED  # m < d
    assert call(desc=lsq.sketch_desc("sjlt", 64, seed=1, s=40)) == lsq.LSQ_ERR_INVALID_ARG
    wide = torch.zeros((1000, 300), dtype=torch.float32, device="cuda")
    assert ctx.pcg_solve_batched([wide], [torch.zeros(1000, dtype=torch.float64, device="cuda")],
                                 [lsq.sketch_desc("sjlt", 1024, seed=1, s=4)],
                                 [torch.zeros(300, dtype=torch.float64, device="cuda")],
                                 raise_on_error=False)[0] == lsq.LSQ_ERR_UNSUPPORTED


def test_batched_gangs(ctx):
    """Problems above the gang size are solved by gangs of 2-4 workgroups (rows split in K blocks, the
    partial sums added in rank order): every problem still meets the oracle bounds, the solutions are
    bitwise equal for any number of workgroups from 4 up (the gang sizes depend on n d alone), and
    within the stop rule's tolerance of the solutions without gangs."""
    from oracle.solve import a_norm_error
    from paper_1911_02675_amd import lsq
    cases = CASES[:6] + CASES[10:]
    ref = None
    try:
        lsq.tune("batched_gang_unit", 65536)  # K = round(n d / 65536) up to 4: gangs for most problems here
        for slots in (0, 4, 7):
            lsq.tune("batched_slots", slots)
            cs = _make(cases)
            st, infos = _run(ctx, cs)
            assert st == 0
            xs = [host(c.x) for c in cs]
            say(f"  gangs, slots {slots}: iters {[i.iters for i in infos]}")
            if ref is None:
                ref = xs
                for c, info in zip(cs, infos):
                    _check_case(c, info)
            else:
                for a, b in zip(ref, xs):
                    assert np.array_equal(a, b)
        # fewer workgroups than a gang needs: refused
        lsq.tune("batched_slots", 3)
        cs = _make([CASES[3]])  # n d = 5.1e6: a gang of 4
        with pytest.raises(lsq.LsqError) as e:
            _run(ctx, cs)
        assert e.value.status == lsq.LSQ_ERR_UNSUPPORTED
    finally:
        lsq.tune("batched_slots", 0)
        lsq.tune("batched_gang_unit", 8 << 20)
    lsq.tune("batched_gang_unit", 0)
    try:
        cs = _make(cases)
        _run(ctx, cs)
        for c, x in zip(cs, ref):
            assert a_norm_error(c.A64, host(c.x), x) <= 3e-10
    finally:
        lsq.tune("batched_gang_unit", 8 << 20)
