"""Thin ctypes binding of libprocmv.so (argument marshalling only).

Every step of the products and the propagation runs in the library's HIP
kernels; PyTorch only provides device memory and the current stream.  If the
library is missing, loading fails loudly: there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprocmv.so")

GEN_PHILOX_GUE = 0
GEN_SINC_DVR = 1
PROCEDURAL, PARTIAL, FULL = 0, 1, 2
FP32, SPLIT_BF16, FP32_COMPENSATED = 0, 1, 2

_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OOM", 3: "INFEASIBLE_PLAN",
           4: "NOT_PLANNED", 5: "HIP", 6: "INTERNAL"}

EXPORTS = [
    "procmv_create_operator", "procmv_plan", "procmv_apply",
    "procmv_spectral_bounds", "procmv_lanczos_bounds", "procmv_cheb_order",
    "procmv_filter_order", "procmv_chebyshev_filter", "procmv_kron_apply", "procmv_kron_propagate",
    "procmv_chebyshev_propagate", "procmv_get_entries", "procmv_selftest_generator",
    "procmv_plan_info",
    "procmv_destroy", "procmv_last_error", "procmv_profile_enable",
    "procmv_profile_read", "procmv_autotune", "procmv_batch_create",
    "procmv_batch_info", "procmv_batch_configure", "procmv_batch_apply",
    "procmv_batch_autotune", "procmv_batch_propagate", "procmv_batch_destroy",
    "procmv_measure", "procmv_plan_candidate_count", "procmv_plan_candidate",
    "procmv_plan_features", "procmv_plan_model_time", "procmv_plan_choose",
    "procmv_plan_auto", "procmv_mlp_param_count", "procmv_mlp_grad",
    "procmv_mlp_train", "procmv_mlp_predict", "procmv_set_tile_shape",
    "procmv_tile_shape_fit", "procmv_apply_noalloc", "procmv_plan_rank",
    "procmv_set_dvr_kernel",
]


class ProcmvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"procmv {_STATUS.get(status, status)}: {msg}")
        self.status = status


class DvrParams(ctypes.Structure):
    _fields_ = [("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
                ("mass", ctypes.c_double), ("omega", ctypes.c_double),
                ("compensate", ctypes.c_int32)]


class MachineModel(ctypes.Structure):
    _fields_ = [("gen_rate", ctypes.c_double * 2), ("dvr_rate", ctypes.c_double),
                ("cache_bw", ctypes.c_double), ("flop_rate", ctypes.c_double),
                ("launch_s", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int64), ("block_size", ctypes.c_int32),
                ("n_blk", ctypes.c_int32), ("n_pair", ctypes.c_int64),
                ("p_cache", ctypes.c_int64), ("cache_bytes", ctypes.c_int64),
                ("work_bytes", ctypes.c_int64), ("strategy", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


_lib = None


def load():
    """Load libprocmv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2606_31598_amd.build`")
    # PyTorch brings its own HIP runtime: it must bring the GPU up before
    # this library's runtime does, or PyTorch later finds no GPU
    import torch
    if torch.cuda.is_available():
        torch.cuda.init()
    L = ctypes.CDLL(LIB_PATH)
    c = ctypes
    vp = c.c_void_p
    L.procmv_create_operator.argtypes = [c.c_int, c.c_uint64, c.c_int64, vp,
                                         c.POINTER(vp)]
    L.procmv_plan.argtypes = [vp, c.c_int32, c.c_int, c.c_double, c.c_int, vp]
    L.procmv_apply.argtypes = [vp, vp, c.c_int64, vp, c.c_int64, c.c_int32, vp]
    L.procmv_apply_noalloc.argtypes = [vp, vp, c.c_int64, vp, c.c_int64, c.c_int32, vp]
    L.procmv_spectral_bounds.argtypes = [vp, c.POINTER(c.c_double),
                                         c.POINTER(c.c_double)]
    L.procmv_cheb_order.argtypes = [c.c_double, c.c_double]
    L.procmv_filter_order.argtypes = [c.c_double, c.c_double]
    L.procmv_kron_apply.argtypes = [vp, c.POINTER(vp), c.c_int32, c.c_int32,
                                    c.POINTER(c.c_double), c.POINTER(c.c_double), c.c_double,
                                    vp, vp, vp]
    L.procmv_kron_propagate.argtypes = [vp, c.POINTER(vp), c.c_int32, c.c_int32,
                                        c.POINTER(c.c_double), c.POINTER(c.c_double),
                                        c.c_double, vp, c.c_double, c.c_int32, c.c_int32,
                                        c.c_double, c.c_double, c.POINTER(c.c_double), vp]
    L.procmv_filter_order.restype = c.c_int32
    L.procmv_chebyshev_filter.argtypes = [vp, vp, c.c_int64, c.c_int32, c.c_double,
                                          c.c_int32, c.c_double, c.c_double,
                                          c.POINTER(c.c_double), vp]
    L.procmv_lanczos_bounds.argtypes = [vp, vp, c.c_int32, c.POINTER(c.c_double),
                                        c.POINTER(c.c_double), c.POINTER(c.c_double),
                                        c.POINTER(c.c_int32), vp]
    L.procmv_cheb_order.restype = c.c_int32
    L.procmv_chebyshev_propagate.argtypes = [vp, vp, c.c_int64, c.c_int32,
                                             c.c_double, c.c_int32, c.c_int32,
                                             c.c_double, c.c_double,
                                             c.POINTER(c.c_double), vp]
    L.procmv_selftest_generator.argtypes = [c.POINTER(c.c_int32), c.POINTER(c.c_int32), vp]
    L.procmv_get_entries.argtypes = [vp, c.c_int64, c.c_int64, c.c_int32,
                                     c.c_int32, vp, vp]
    L.procmv_plan_info.argtypes = [vp, c.POINTER(PlanInfo)]
    L.procmv_profile_enable.argtypes = [vp, c.c_int32]
    L.procmv_profile_read.argtypes = [vp, c.POINTER(c.c_double),
                                      c.POINTER(c.c_int64),
                                      c.POINTER(c.c_double),
                                      c.POINTER(c.c_int64)]
    L.procmv_autotune.argtypes = [vp, c.c_int32, c.c_int32, vp,
                                  c.POINTER(c.c_int32), c.POINTER(c.c_double)]
    L.procmv_batch_create.argtypes = [c.POINTER(vp), c.c_int32, c.c_int32,
                                      c.POINTER(vp)]
    L.procmv_batch_info.argtypes = [vp, c.POINTER(c.c_int64), c.POINTER(c.c_int64),
                                    c.POINTER(c.c_int32), c.POINTER(c.c_int32),
                                    c.POINTER(c.c_int32)]
    L.procmv_batch_configure.argtypes = [vp, c.c_int32, c.c_int32, c.c_int32]
    L.procmv_batch_apply.argtypes = [vp, vp, vp, vp]
    L.procmv_batch_autotune.argtypes = [vp, vp, vp, c.c_int32, vp,
                                        c.POINTER(c.c_double)]
    L.procmv_batch_propagate.argtypes = [vp, vp, c.c_double, c.c_int32,
                                         c.c_int32, c.c_double, c.c_double,
                                         c.c_int32, c.POINTER(c.c_double), vp]
    L.procmv_measure.argtypes = [c.c_int, c.c_uint64, c.c_int64, vp, c.c_int32,
                                 c.c_int32, c.c_int, c.c_double, c.c_int, c.c_int32,
                                 c.c_int32, vp, c.POINTER(c.c_double),
                                 c.POINTER(c.c_double)]
    f32p = c.POINTER(c.c_float)
    i32p = c.POINTER(c.c_int32)
    f64p = c.POINTER(c.c_double)
    L.procmv_plan_candidate_count.restype = c.c_int32
    L.procmv_plan_candidate.argtypes = [c.c_int32, i32p, i32p, f64p]
    L.procmv_plan_features.argtypes = [c.c_int64, c.c_int32, c.c_double, c.c_int64,
                                       c.c_int32, c.c_int32, c.c_int32, c.c_double,
                                       f32p, f64p, i32p]
    L.procmv_plan_model_time.argtypes = [c.POINTER(MachineModel), c.c_int64, c.c_int32,
                                         c.c_int32, c.c_int32, c.c_int32, c.c_double,
                                         c.c_int64, f64p, f64p]
    L.procmv_plan_choose.argtypes = [c.c_int32, c.POINTER(MachineModel), f32p, f32p,
                                     c.c_int64, c.c_int32, c.c_double, c.c_int64,
                                     c.c_int32, i32p, f64p]
    L.procmv_plan_rank.argtypes = [c.c_int32, c.POINTER(MachineModel), f32p, f32p,
                                   c.c_int64, c.c_int32, c.c_double, c.c_int64,
                                   c.c_int32, i32p, f64p, i32p]
    L.procmv_plan_auto.argtypes = [vp, c.c_int32, c.c_double, c.c_int64, c.c_int32,
                                   c.POINTER(MachineModel), f32p, f32p, vp, i32p]
    L.procmv_set_tile_shape.argtypes = [vp, c.c_int32]
    L.procmv_set_dvr_kernel.argtypes = [vp, c.c_int32]
    L.procmv_tile_shape_fit.argtypes = [c.c_int32, c.c_int32, c.c_int64, c.c_int32]
    L.procmv_tile_shape_fit.restype = c.c_int32
    L.procmv_mlp_param_count.restype = c.c_int32
    L.procmv_mlp_grad.argtypes = [f32p, f32p, f32p, c.c_int32, f32p, f32p]
    L.procmv_mlp_train.argtypes = [f32p, f32p, c.c_int32, c.c_int32, c.c_float, f32p, f32p]
    L.procmv_mlp_predict.argtypes = [f32p, f32p, c.c_int32, f32p]
    L.procmv_batch_destroy.argtypes = [vp]
    L.procmv_batch_destroy.restype = None
    L.procmv_destroy.argtypes = [vp]
    L.procmv_destroy.restype = None
    L.procmv_last_error.restype = c.c_char_p
    for name in EXPORTS:
        if name in ("procmv_cheb_order", "procmv_destroy", "procmv_last_error",
                    "procmv_batch_destroy", "procmv_plan_candidate_count",
                    "procmv_mlp_param_count", "procmv_tile_shape_fit"):
            continue
        getattr(L, name).restype = c.c_int
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise ProcmvError(status, load().procmv_last_error().decode())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _vec_arg(t, D):
    """(pointer, leading dimension, nvec) of a (nvec, D) complex64 CUDA tensor."""
    import torch
    if t.dtype != torch.complex64 or not t.is_cuda:
        raise TypeError("vectors must be complex64 CUDA tensors")
    if t.dim() == 1:
        t = t.unsqueeze(0)
    if t.dim() != 2 or t.shape[1] != D or t.stride(1) != 1:
        raise ValueError(f"expected shape (nvec, {D}) with unit column stride")
    return ctypes.c_void_p(t.data_ptr()), t.stride(0) if t.shape[0] > 1 else D, t.shape[0]


def cheb_order(x: float, tol: float = 1e-10) -> int:
    return int(load().procmv_cheb_order(float(x), float(tol)))


def _kron_args(HB, Bs, HS, As, tensors):
    import torch
    HS = np.ascontiguousarray(HS, np.complex128)
    dS = HS.shape[0]
    As = np.ascontiguousarray(np.asarray(As, np.complex128).reshape(-1, dS, dS))
    if As.shape[0] != len(Bs):
        raise ValueError("one A per bath operator")
    for t in tensors:
        if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous() \
                or tuple(t.shape) != (dS, HB.D):
            raise ValueError(f"state tensors must be contiguous complex64 CUDA ({dS}, {HB.D})")
    handles = (ctypes.c_void_p * max(len(Bs), 1))(*[b._h.value for b in Bs])
    dp = ctypes.POINTER(ctypes.c_double)
    return (HB._h, ctypes.cast(handles, ctypes.POINTER(ctypes.c_void_p)), len(Bs), dS,
            HS.view(np.float64).ctypes.data_as(dp),
            As.view(np.float64).ctypes.data_as(dp) if len(Bs) else None), (HS, As, handles)


def kron_apply(HB, Bs, HS, As, g, X, Y, stream=None):
    """Y = (H_S x I + I x H_B + g sum_a A_a x B_a) X for the (d_S, d_B)
    complex64 CUDA tensors X, Y (row s = system index s).  HB and Bs are
    planned Operators of the same D = d_B; HS (d_S, d_S) and As (n_int, d_S,
    d_S) are host complex matrices."""
    args, keep = _kron_args(HB, Bs, HS, As, (X, Y))
    _check(load().procmv_kron_apply(*args, float(g), ctypes.c_void_p(X.data_ptr()),
                                    ctypes.c_void_p(Y.data_ptr()), _stream(stream)))


def kron_propagate(HB, Bs, HS, As, g, psi, dt, nsteps, c, R, K=0, norms=False,
                   stream=None):
    """psi <- exp(-i H dt)^nsteps psi in place for the system-bath operator of
    ``kron_apply`` (centered Chebyshev with centre c and half-width R);
    returns the binary64 norm after each step when ``norms``."""
    args, keep = _kron_args(HB, Bs, HS, As, (psi,))
    out = np.zeros(max(int(nsteps), 1), np.float64) if norms else None
    optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if norms else None
    _check(load().procmv_kron_propagate(*args, float(g), ctypes.c_void_p(psi.data_ptr()),
                                        float(dt), int(K), int(nsteps), float(c), float(R),
                                        optr, _stream(stream)))
    return out


def tile_shape_fit(nvec, shape, D, cache_block=0) -> int:
    """VALU tile shape launched for a requested shape (see the header)."""
    return int(load().procmv_tile_shape_fit(int(nvec), int(shape), int(D), int(cache_block)))


def filter_order(z: float, tol: float = 1e-10) -> int:
    return int(load().procmv_filter_order(float(z), float(tol)))


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def selftest_generator(stream=None):
    """(logarithm, square-root) bitwise mismatches of the generator's short
    division and square root against IEEE, over all 2^23 uniforms."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(load().procmv_selftest_generator(ctypes.byref(a), ctypes.byref(b), _stream(stream)))
    return a.value, b.value


def plan_candidates():
    """[(block_size, strategy, cache_fraction)] in candidate-index order."""
    L = load()
    out = []
    for q in range(L.procmv_plan_candidate_count()):
        b, st, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(L.procmv_plan_candidate(q, ctypes.byref(b), ctypes.byref(st), ctypes.byref(f)))
        out.append((b.value, st.value, f.value))
    return out


def plan_features(D, nvec, budget_bytes, reuse, family, b, strategy, f):
    """(8 features, M_tot bytes, feasible) of a (problem, plan) pair."""
    x = np.zeros(8, np.float32)
    mt, fe = ctypes.c_double(), ctypes.c_int32()
    _check(load().procmv_plan_features(int(D), int(nvec), float(budget_bytes), int(reuse),
                                       int(family), int(b), int(strategy), float(f),
                                       x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                       ctypes.byref(mt), ctypes.byref(fe)))
    return x, mt.value, bool(fe.value)


def plan_model_time(mm, D, nvec, family, b, strategy, f, reuse):
    tf, ta = ctypes.c_double(), ctypes.c_double()
    _check(load().procmv_plan_model_time(ctypes.byref(mm), int(D), int(nvec), int(family),
                                         int(b), int(strategy), float(f), int(reuse),
                                         ctypes.byref(tf), ctypes.byref(ta)))
    return tf.value, ta.value


def plan_choose(planner, D, nvec, budget_bytes, reuse, family, mm=None, params=None,
                norm=None):
    """Index of the chosen candidate (planner 0 analytic, 1 learned)."""
    idx, sc = ctypes.c_int32(), ctypes.c_double()
    pa = _f32(params) if params is not None else (None, None)
    na = _f32(norm) if norm is not None else (None, None)
    pp, nn = pa[1], na[1]
    _check(load().procmv_plan_choose(int(planner), ctypes.byref(mm) if mm is not None else None,
                                     pp, nn, int(D), int(nvec), float(budget_bytes), int(reuse),
                                     int(family), ctypes.byref(idx), ctypes.byref(sc)))
    return idx.value, sc.value


def plan_rank(planner, D, nvec, budget_bytes, reuse, family, mm=None, params=None,
              norm=None):
    """Feasible candidates best first: ([index], [score]) (planner 0
    analytic, 1 learned)."""
    nc = load().procmv_plan_candidate_count()
    order = np.zeros(nc, np.int32)
    score = np.zeros(nc, np.float64)
    n = ctypes.c_int32()
    pa = _f32(params) if params is not None else (None, None)
    na = _f32(norm) if norm is not None else (None, None)
    _check(load().procmv_plan_rank(int(planner), ctypes.byref(mm) if mm is not None else None,
                                   pa[1], na[1], int(D), int(nvec), float(budget_bytes),
                                   int(reuse), int(family),
                                   order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   score.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(n)))
    return order[:n.value].tolist(), score[:n.value].tolist()


def mlp_param_count():
    return int(load().procmv_mlp_param_count())


def mlp_grad(params, z, t):
    """Gradient and loss of one GPU forward/backward pass (test hook)."""
    p, pp = _f32(params)
    zz, zp = _f32(z)
    tt, tp = _f32(t)
    g = np.zeros(mlp_param_count(), np.float32)
    loss = np.zeros(1, np.float32)
    _check(load().procmv_mlp_grad(pp, zp, tp, int(tt.size),
                                  g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                  loss.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return g, float(loss[0])


def mlp_train(z, t, params, epochs, lr):
    """Full-batch Adam on the GPU; returns (params, loss history)."""
    zz, zp = _f32(z)
    tt, tp = _f32(t)
    p = np.array(params, dtype=np.float32, copy=True)
    hist = np.zeros(max(epochs, 1), np.float32)
    _check(load().procmv_mlp_train(zp, tp, int(tt.size), int(epochs), float(lr),
                                   p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   hist.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return p, hist[:epochs]


def mlp_predict(params, z):
    p, pp = _f32(params)
    zz, zp = _f32(z)
    y = np.zeros(zz.shape[0], np.float32)
    _check(load().procmv_mlp_predict(pp, zp, int(zz.shape[0]),
                                     y.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return y


def measure(gen, D, nvec, block_size, strategy, cache_fraction=0.0,
            precision=FP32, seed=1, warmup=1, reps=2, stream=None):
    """Library-measured (t_fill_ms, t_apply_ms) of one operator and plan;
    None when the plan does not fit in device memory."""
    tf, ta = ctypes.c_double(), ctypes.c_double()
    st = load().procmv_measure(gen, ctypes.c_uint64(seed), int(D), None, int(nvec),
                               int(block_size), int(strategy), float(cache_fraction),
                               int(precision), int(warmup), int(reps), _stream(stream),
                               ctypes.byref(tf), ctypes.byref(ta))
    if st == 2:
        return None
    _check(st)
    return tf.value, ta.value


class Operator:
    """A dense Hermitian operator applied without materialising its matrix."""

    def __init__(self, gen, D, seed=0, x_min=-20.0, x_max=20.0, mass=1.0,
                 omega=1.0, compensate=True):
        L = load()
        self.D = int(D)
        self.gen = gen
        h = ctypes.c_void_p()
        params = None
        if gen == GEN_SINC_DVR:
            self._params = DvrParams(x_min, x_max, mass, omega, 1 if compensate else 0)
            params = ctypes.byref(self._params)
        _check(L.procmv_create_operator(gen, ctypes.c_uint64(seed), self.D,
                                        params, ctypes.byref(h)))
        self._h = h

    @classmethod
    def gue(cls, D, seed):
        return cls(GEN_PHILOX_GUE, D, seed=seed)

    @classmethod
    def dvr(cls, D, **kw):
        return cls(GEN_SINC_DVR, D, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().procmv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def plan(self, block_size=256, strategy=PROCEDURAL, cache_fraction=0.0,
             precision=FP32, stream=None):
        _check(load().procmv_plan(self._h, int(block_size), int(strategy),
                                  float(cache_fraction), int(precision),
                                  _stream(stream)))
        return self

    def plan_auto(self, nvec, budget_bytes, reuse, planner=1, mm=None, params=None,
                  norm=None, stream=None):
        """Choose the plan with the analytic (0), learned (1), measured (2:
        analytic top-K timed) or hybrid (3: learned top-K timed) planner and
        apply it (binary32); returns the chosen candidate index."""
        idx = ctypes.c_int32()
        pa = _f32(params) if params is not None else (None, None)   # keep the arrays alive
        na = _f32(norm) if norm is not None else (None, None)
        _check(load().procmv_plan_auto(self._h, int(nvec), float(budget_bytes), int(reuse),
                                       int(planner),
                                       ctypes.byref(mm) if mm is not None else None,
                                       pa[1], na[1], _stream(stream), ctypes.byref(idx)))
        return idx.value

    def plan_info(self) -> dict:
        info = PlanInfo()
        _check(load().procmv_plan_info(self._h, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in PlanInfo._fields_}

    def apply(self, X, Y=None, stream=None):
        """Y = H X for a (nvec, D) complex64 CUDA tensor X."""
        import torch
        px, ldx, nv = _vec_arg(X, self.D)
        if Y is None:
            Y = torch.empty((nv, self.D), dtype=torch.complex64, device=X.device)
        py, ldy, nvy = _vec_arg(Y, self.D)
        if nvy != nv:
            raise ValueError("X and Y hold different numbers of vectors")
        _check(load().procmv_apply(self._h, px, ldx, py, ldy, nv, _stream(stream)))
        return Y

    def spectral_bounds(self):
        c = ctypes.c_double()
        R = ctypes.c_double()
        _check(load().procmv_spectral_bounds(self._h, ctypes.byref(c), ctypes.byref(R)))
        return c.value, R.value

    def lanczos_bounds(self, v0, m=40, stream=None):
        """Matrix-free Lanczos spectral bounds from the start vector ``v0``
        (complex64 CUDA tensor of D entries): dict with E_min, E_max, the
        extreme Ritz values, their residual estimates, c, R and the recurrence
        coefficients (binary64)."""
        pp, _, nv = _vec_arg(v0, self.D)
        if nv != 1:
            raise ValueError("one start vector")
        out = np.zeros(6, np.float64)
        al = np.zeros(max(int(m), 1), np.float64)
        be = np.zeros(max(int(m), 1), np.float64)
        n = ctypes.c_int32()
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load().procmv_lanczos_bounds(
            self._h, pp, int(m), out.ctypes.data_as(dp), al.ctypes.data_as(dp),
            be.ctypes.data_as(dp), ctypes.byref(n), _stream(stream)))
        k = n.value
        return {"e_min": out[0], "e_max": out[1], "theta_min": out[2], "theta_max": out[3],
                "r_min": out[4], "r_max": out[5], "c": 0.5 * (out[1] + out[0]),
                "R": 0.5 * (out[1] - out[0]), "steps": k, "alpha": al[:k], "beta": be[:k]}

    def filter(self, psi, tau, K=0, c=0.0, R=0.0, norms=False, stream=None):
        """psi <- exp(-tau H) psi in place (imaginary-time Chebyshev filter,
        not normalised); returns the (nvec,) binary64 norms when ``norms``."""
        pp, ld, nv = _vec_arg(psi, self.D)
        out = np.zeros(nv, np.float64) if norms else None
        optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if norms else None
        _check(load().procmv_chebyshev_filter(
            self._h, pp, ld, nv, float(tau), int(K), float(c), float(R), optr,
            _stream(stream)))
        return out

    def propagate(self, psi, dt, nsteps=1, K=0, c=0.0, R=0.0, norms=False,
                  stream=None):
        """psi <- exp(-i H dt)^nsteps psi in place (Chebyshev); returns the
        (nsteps, nvec) binary64 norms when ``norms``."""
        pp, ld, nv = _vec_arg(psi, self.D)
        out = np.zeros((max(nsteps, 1), nv), np.float64) if norms else None
        optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if norms else None
        _check(load().procmv_chebyshev_propagate(
            self._h, pp, ld, nv, float(dt), int(K), int(nsteps), float(c),
            float(R), optr, _stream(stream)))
        return out

    def profile(self, every=1):
        """Time every ``every``-th tile / reduction launch with HIP events
        (0 switches it off)."""
        _check(load().procmv_profile_enable(self._h, int(every)))

    def profile_read(self) -> dict:
        """Summed event durations (ms) and counts of the timed launches."""
        tm, rm = ctypes.c_double(), ctypes.c_double()
        tn, rn = ctypes.c_int64(), ctypes.c_int64()
        _check(load().procmv_profile_read(self._h, ctypes.byref(tm), ctypes.byref(tn),
                                          ctypes.byref(rm), ctypes.byref(rn)))
        return {"tile_ms": tm.value, "tile_n": tn.value,
                "reduce_ms": rm.value, "reduce_n": rn.value}

    def autotune(self, nvec=1, reps=3, stream=None):
        """Measure the VALU tile shapes and keep the fastest; returns
        (shape, ms per product)."""
        sh, ms = ctypes.c_int32(), ctypes.c_double()
        _check(load().procmv_autotune(self._h, int(nvec), int(reps), _stream(stream),
                                      ctypes.byref(sh), ctypes.byref(ms)))
        return sh.value, ms.value

    def set_dvr_kernel(self, kind):
        """Procedural sinc-DVR product kernel: 0 automatic, 1 VALU Toeplitz
        kernel, 2 binary32 matrix-core Toeplitz kernel, 3 split-bf16
        matrix-core Toeplitz kernel (2 and 3: one vector per launch)."""
        _check(load().procmv_set_dvr_kernel(self._h, int(kind)))
        return self

    def set_tile_shape(self, shape):
        _check(load().procmv_set_tile_shape(self._h, int(shape)))
        return self

    def entries(self, r0, c0, nr, nc, stream=None):
        """Generated binary32 entries of a window, as a complex64 CUDA tensor."""
        import torch
        out = torch.empty((nr, nc), dtype=torch.complex64, device="cuda")
        _check(load().procmv_get_entries(self._h, int(r0), int(c0), int(nr),
                                         int(nc), ctypes.c_void_p(out.data_ptr()),
                                         _stream(stream)))
        return out


class Batch:
    """Independent operators applied together in one persistent launch.

    Vectors are packed: instance k's ``nvec`` vectors of length D_k start at
    element ``offsets[k]`` of one complex64 buffer of ``total`` elements.
    """

    def __init__(self, ops, nvec):
        L = load()
        self.ops = list(ops)            # keep the operators alive
        self.nvec = int(nvec)
        arr = (ctypes.c_void_p * len(self.ops))(*[o._h.value for o in self.ops])
        h = ctypes.c_void_p()
        _check(L.procmv_batch_create(arr, len(self.ops), self.nvec, ctypes.byref(h)))
        self._h = h
        sizes = np.array([o.D for o in self.ops], dtype=np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.nvec * sizes)[:-1]])
        self.total = int(self.nvec * sizes.sum())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().procmv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        t, it = ctypes.c_int64(), ctypes.c_int64()
        sh, g, o = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().procmv_batch_info(self._h, ctypes.byref(t), ctypes.byref(it),
                                        ctypes.byref(sh), ctypes.byref(g), ctypes.byref(o)))
        return {"total": t.value, "items": it.value, "shape": sh.value,
                "grid": g.value, "order": o.value}

    def configure(self, shape, grid, order):
        _check(load().procmv_batch_configure(self._h, int(shape), int(grid), int(order)))

    def _ptr(self, t):
        import torch
        if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous() \
                or t.numel() != self.total:
            raise ValueError(f"expected a contiguous complex64 CUDA tensor of {self.total} elements")
        return ctypes.c_void_p(t.data_ptr())

    def apply(self, X, Y, stream=None):
        _check(load().procmv_batch_apply(self._h, self._ptr(X), self._ptr(Y), _stream(stream)))
        return Y

    def autotune(self, X, Y, reps=3, stream=None):
        ms = ctypes.c_double()
        _check(load().procmv_batch_autotune(self._h, self._ptr(X), self._ptr(Y), int(reps),
                                            _stream(stream), ctypes.byref(ms)))
        return ms.value

    def propagate(self, psi, dt, nsteps, c, R, K=0, graph=True, norms=False, stream=None):
        out = np.zeros(len(self.ops) * self.nvec) if norms else None
        optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if norms else None
        _check(load().procmv_batch_propagate(self._h, self._ptr(psi), float(dt), int(K),
                                             int(nsteps), float(c), float(R),
                                             1 if graph else 0, optr, _stream(stream)))
        return out
