"""Thin ctypes binding of liblsq (include/lsq.h).  Argument marshalling only: every step of the
computation runs in the HIP library; torch tensors are used for device memory and streams.

The library must have been built (python -m paper_1911_02675_amd.build); importing this module on a
machine without it raises, and there is no fallback implementation.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsq.so")

LSQ_OK, LSQ_ERR_INVALID_ARG, LSQ_ERR_RANK, LSQ_ERR_NOT_CONVERGED = 0, 1, 2, 3
LSQ_ERR_NONFINITE, LSQ_ERR_HIP, LSQ_ERR_NOMEM, LSQ_ERR_UNSUPPORTED = 4, 5, 6, 7
LSQ_F64, LSQ_F32, LSQ_BF16 = 0, 1, 2
LSQ_GAUSSIAN, LSQ_SRHT, LSQ_SJLT, LSQ_HAAR = 0, 1, 2, 3
KINDS = {"gaussian": LSQ_GAUSSIAN, "srht": LSQ_SRHT, "sjlt": LSQ_SJLT, "haar": LSQ_HAAR}
DTYPES = {"f64": LSQ_F64, "f32": LSQ_F32, "bf16": LSQ_BF16}

EXPORTED = [
    "lsq_create", "lsq_destroy", "lsq_sketch", "lsq_factor", "lsq_fused_pass", "lsq_pcg_solve",
    "lsq_ihs_solve", "lsq_fcg_solve", "lsq_pcg_solve_batched", "lsq_draw_srht", "lsq_draw_sjlt", "lsq_draw_gaussian",
    "lsq_fused_pass_noalloc", "lsq_fused_pass_timing", "lsq_read_bandwidth", "lsq_copy_bandwidth", "lsq_choose_sketch_size", "lsq_tune", "lsq_set_option", "lsq_status_string", "lsq_last_error", "lsq_version",
]


class Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int64), ("lda", C.c_int64), ("a_dtype", C.c_int32),
                ("pad_", C.c_int32), ("A", C.c_void_p), ("y", C.c_void_p)]


class SketchDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("s", C.c_int32), ("m", C.c_int64), ("compute", C.c_int32),
                ("pad_", C.c_int32), ("seed", C.c_uint64), ("t", C.c_uint64)]


class PcgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("stop_rule", C.c_int32),
                ("mixed", C.c_int32), ("max_refine", C.c_int32), ("inner_f32", C.c_int32),
                ("check_every", C.c_int32), ("x_ref", C.c_void_p)]


class IhsOpts(C.Structure):
    _fields_ = [("mu", C.c_double), ("beta", C.c_double), ("iters", C.c_int32), ("refresh", C.c_int32),
                ("mu_rule", C.c_int32), ("pad_", C.c_int32), ("x_ref", C.c_void_p)]


class FcgOpts(C.Structure):
    _fields_ = [("iters", C.c_int32), ("window", C.c_int32), ("refresh", C.c_int32), ("pad_", C.c_int32),
                ("x_ref", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refinements", C.c_int32), ("est_rel_err", C.c_double),
                ("t_sketch_ms", C.c_double), ("t_factor_ms", C.c_double), ("t_iter_ms", C.c_double),
                ("t_total_ms", C.c_double), ("bytes_streamed", C.c_double), ("mu", C.c_double),
                ("status", C.c_int32), ("pad_", C.c_int32), ("t_start_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MsizeEntry(C.Structure):
    _fields_ = [("m", C.c_int64), ("iters", C.c_int32), ("pad_", C.c_int32), ("t_sketch_ms", C.c_double),
                ("t_factor_ms", C.c_double), ("predicted_ms", C.c_double), ("r_spread", C.c_double)]


class LsqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)} ({status}): {msg}")
        self.status = status


_lib = None


def load():
    """Load liblsq.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} not found: run python -m paper_1911_02675_amd.build")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "lsq_create": ([C.POINTER(C.c_void_p), P], I32),
        "lsq_destroy": ([P], None),
        "lsq_sketch": ([P, C.POINTER(Problem), C.POINTER(SketchDesc), P, I64, I32], I32),
        "lsq_factor": ([P, P, I64, I64, I64, P, P], I32),
        "lsq_fused_pass": ([P, C.POINTER(Problem), I32, I32, P, P, P], I32),
        "lsq_fused_pass_noalloc": ([P, C.POINTER(Problem), I32, I32, P, P, P], I32),
        "lsq_pcg_solve": ([P, C.POINTER(Problem), C.POINTER(SketchDesc), C.POINTER(PcgOpts), P, P,
                           C.POINTER(Info)], I32),
        "lsq_ihs_solve": ([P, C.POINTER(Problem), C.POINTER(SketchDesc), C.POINTER(IhsOpts), P, P,
                           C.POINTER(Info)], I32),
        "lsq_fcg_solve": ([P, C.POINTER(Problem), C.POINTER(SketchDesc), C.POINTER(FcgOpts), P, P,
                           C.POINTER(Info)], I32),
        "lsq_pcg_solve_batched": ([P, I32, C.POINTER(Problem), C.POINTER(SketchDesc),
                                   C.POINTER(PcgOpts), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.POINTER(Info)], I32),
        "lsq_draw_srht": ([P, U64, U64, I64, I64, P, P], I32),
        "lsq_draw_sjlt": ([P, U64, U64, I64, I64, I32, P, P], I32),
        "lsq_draw_gaussian": ([P, U64, U64, I64, I64, I64, P], I32),
        "lsq_fused_pass_timing": ([P, I32, C.POINTER(D), C.POINTER(D), C.POINTER(I64)], I32),
        "lsq_read_bandwidth": ([P, P, I64, I32, C.POINTER(D)], I32),
        "lsq_copy_bandwidth": ([P, P, P, I64, I32, C.POINTER(D)], I32),
        "lsq_choose_sketch_size": ([P, C.POINTER(Problem), C.POINTER(SketchDesc), D, D, I32, C.POINTER(MsizeEntry),
                                    I32, C.POINTER(I32), C.POINTER(I64), C.POINTER(D)], I32),
        "lsq_tune": ([C.c_char_p, I64], I32),
        "lsq_set_option": ([P, C.c_char_p, I64], I32),
        "lsq_status_string": ([I32], C.c_char_p),
        "lsq_last_error": ([], C.c_char_p),
        "lsq_version": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def status_string(s):
    return load().lsq_status_string(s).decode()


def _check(status):
    if status != LSQ_OK:
        raise LsqError(status, load().lsq_last_error().decode())
    return status


def tune(key, value):
    """Set a process-wide launch parameter of the library (see lsq_tune in include/lsq.h)."""
    _check(load().lsq_tune(key.encode(), int(value)))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def problem(A, y):
    """lsq_problem for a row-major torch tensor A (float64 or float32, n x d, unit column stride) and
    float64 y on the device."""
    import torch
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be 2-D with unit column stride")
    if A.dtype == torch.float64:
        dt = LSQ_F64
    elif A.dtype == torch.float32:
        dt = LSQ_F32
    else:
        raise ValueError("A must be float64 or float32")
    if y.dtype != torch.float64 or y.numel() != A.shape[0]:
        raise ValueError("y must be float64 with n entries")
    p = Problem(A.shape[0], A.shape[1], A.stride(0), dt, 0, A.data_ptr(), y.data_ptr())
    p._keep = (A, y)
    return p


def sketch_desc(kind, m, seed=0, t=0, s=1, compute="f64"):
    return SketchDesc(KINDS[kind], s, m, DTYPES[compute], 0, seed, t)


class Context:
    """An lsq_ctx bound to the current device and torch's current stream (or `stream`)."""

    def __init__(self, stream=None):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        _check(self.lib.lsq_create(C.byref(h), C.c_void_p(stream.cuda_stream)))
        self.h = h

    def close(self):
        if self.h:
            self.lib.lsq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- entry points (same names as the C ABI, without the prefix) ----
    def set_option(self, key, value):
        """A numerics option of this context ("factor", "srht_passb"; see lsq_set_option)."""
        _check(self.lib.lsq_set_option(self.h, key.encode(), int(value)))

    def sketch(self, A, y, desc, SA):
        p = problem(A, y)
        _check(self.lib.lsq_sketch(self.h, C.byref(p), C.byref(desc), _ptr(SA), SA.stride(0), LSQ_F64))
        return SA

    def factor(self, SA, R=None, W=None):
        m, d = SA.shape
        _check(self.lib.lsq_factor(self.h, _ptr(SA), m, d, SA.stride(0), _ptr(R), _ptr(W)))
        return R, W

    def fused_pass(self, A, y, v, w, scal, mode=0, f32_math=False):
        p = problem(A, y)
        _check(self.lib.lsq_fused_pass(self.h, C.byref(p), mode, int(f32_math), _ptr(v), _ptr(w),
                                       _ptr(scal)))

    def fused_pass_noalloc(self, A, y, v, w, scal, mode=0, f32_math=False):
        """Queued on the context's stream; the caller synchronises."""
        p = problem(A, y)
        _check(self.lib.lsq_fused_pass_noalloc(self.h, C.byref(p), mode, int(f32_math), _ptr(v), _ptr(w),
                                               _ptr(scal)))

    def pcg_solve(self, A, y, desc, x, tol=1e-10, max_iter=200, stop_rule=0, mixed=0, max_refine=8,
                  inner_f32=0, check_every=8, x_ref=None, err_trace=None, raise_on_error=True):
        p = problem(A, y)
        o = PcgOpts(tol, max_iter, stop_rule, mixed, max_refine, inner_f32, check_every,
                    None if x_ref is None else x_ref.data_ptr())
        info = Info()
        st = self.lib.lsq_pcg_solve(self.h, C.byref(p), C.byref(desc), C.byref(o), _ptr(x),
                                    _ptr(err_trace), C.byref(info))
        if raise_on_error:
            _check(st)
        return st, info

    def ihs_solve(self, A, y, desc, x, iters=20, mu=0.0, beta=0.0, refresh=1, mu_rule=0, x_ref=None,
                  err_trace=None):
        p = problem(A, y)
        o = IhsOpts(mu, beta, iters, refresh, mu_rule, 0, None if x_ref is None else x_ref.data_ptr())
        info = Info()
        _check(self.lib.lsq_ihs_solve(self.h, C.byref(p), C.byref(desc), C.byref(o), _ptr(x),
                                      _ptr(err_trace), C.byref(info)))
        return info

    def fcg_solve(self, A, y, desc, x, iters=20, window=1, refresh=1, x_ref=None, err_trace=None):
        """Flexible CG: window 0 = line-searched IHS, 1 = IPCG, >= iters = GCC."""
        p = problem(A, y)
        o = FcgOpts(iters, window, refresh, 0, None if x_ref is None else x_ref.data_ptr())
        info = Info()
        _check(self.lib.lsq_fcg_solve(self.h, C.byref(p), C.byref(desc), C.byref(o), _ptr(x),
                                      _ptr(err_trace), C.byref(info)))
        return info

    def pcg_solve_batched(self, As, ys, descs, xs, tol=1e-10, max_iter=200, mixed=1, max_refine=8,
                          Rs=None, raise_on_error=True):
        """Solve len(As) independent problems in one persistent launch (SJLT descriptors).  Returns
        (status, list of Info); xs (and Rs entries that are not None) are written on the device."""
        n = len(As)
        probs = (Problem * n)(*[problem(A, y) for A, y in zip(As, ys)])
        ds = (SketchDesc * n)(*descs)
        xp = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        rp = None
        if Rs is not None:
            rp = (C.c_void_p * n)(*[None if R is None else R.data_ptr() for R in Rs])
        infos = (Info * n)()
        o = PcgOpts(tol, max_iter, 0, mixed, max_refine, 0, 8, None)
        st = self.lib.lsq_pcg_solve_batched(self.h, n, probs, ds, C.byref(o), xp, rp, infos)
        if raise_on_error:
            _check(st)
        return st, list(infos)

    def draw_srht(self, seed, t, N, m, signs=None, rows=None):
        _check(self.lib.lsq_draw_srht(self.h, seed, t, N, m, _ptr(signs), _ptr(rows)))

    def draw_sjlt(self, seed, t, n, m, s, targets, signs):
        _check(self.lib.lsq_draw_sjlt(self.h, seed, t, n, m, s, _ptr(targets), _ptr(signs)))

    def draw_gaussian(self, seed, t, m, j0, ncols, G):
        _check(self.lib.lsq_draw_gaussian(self.h, seed, t, m, j0, ncols, _ptr(G)))

    def choose_sketch_size(self, A, y, desc, tol=1e-10, extra_passes=0.0, reps=2):
        """Section 6's chooser with this GPU's measured costs (lsq_choose_sketch_size).  Returns
        (m_best, table, t_pass_ms) with table a list of dicts (m, iters, t_sketch_ms, t_factor_ms,
        predicted_ms, r_spread)."""
        p = problem(A, y)
        tab = (MsizeEntry * 16)()
        cnt, mb, tp = C.c_int32(), C.c_int64(), C.c_double()
        _check(self.lib.lsq_choose_sketch_size(self.h, C.byref(p), C.byref(desc), tol, extra_passes, reps, tab, 16,
                                               C.byref(cnt), C.byref(mb), C.byref(tp)))
        rows = [{k: getattr(tab[i], k) for k, _ in MsizeEntry._fields_ if k != "pad_"} for i in range(cnt.value)]
        return mb.value, rows, tp.value

    def copy_bandwidth(self, src, dst, reps=5):
        """Measured read + write ceiling (GB/s, both directions) copying src to dst (see lsq_copy_bandwidth)."""
        g = C.c_double()
        nb = min(src.numel() * src.element_size(), dst.numel() * dst.element_size())
        _check(self.lib.lsq_copy_bandwidth(self.h, _ptr(src), _ptr(dst), nb, reps, C.byref(g)))
        return g.value

    def read_bandwidth(self, buf, reps=5):
        """Measured read ceiling (GB/s) over the device tensor buf (see lsq_read_bandwidth)."""
        g = C.c_double()
        _check(self.lib.lsq_read_bandwidth(self.h, _ptr(buf), buf.numel() * buf.element_size(), reps,
                                           C.byref(g)))
        return g.value

    def fused_pass_timing(self, reset=False):
        last, avg, cnt = C.c_double(), C.c_double(), C.c_int64()
        _check(self.lib.lsq_fused_pass_timing(self.h, int(reset), C.byref(last), C.byref(avg),
                                              C.byref(cnt)))
        return last.value, avg.value, cnt.value
