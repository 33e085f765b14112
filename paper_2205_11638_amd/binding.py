"""Thin ctypes binding of libdd.so: argument marshalling only.

Every step of the solver runs in the library's HIP kernels; this module passes
pointers, sizes and the current torch stream.  It fails loudly when the built
library is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# DD_SANITIZE=1 loads the host-sanitized build (CPU checks only; see build.py)
LIB_PATH = os.path.join(HERE, "libdd_san.so" if os.environ.get("DD_SANITIZE") == "1" else "libdd.so")

DD_OK, DD_E_ARG, DD_E_INFEASIBLE, DD_E_FORCED, DD_E_PARAM, DD_E_HIP, DD_E_UNSUPPORTED, DD_E_OOM, DD_E_NONFINITE, \
    DD_E_STATE, DD_E_CHECKPOINT = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10

_NAMES = {0: "DD_OK", -1: "DD_E_ARG", -2: "DD_E_INFEASIBLE", -3: "DD_E_FORCED", -4: "DD_E_PARAM", -5: "DD_E_HIP",
          -6: "DD_E_UNSUPPORTED", -7: "DD_E_OOM", -8: "DD_E_NONFINITE", -9: "DD_E_STATE", -10: "DD_E_CHECKPOINT"}


class DDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class dd_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("c", C.POINTER(C.c_double)), ("m", C.c_int32),
                ("row_ptr", C.POINTER(C.c_int64)), ("col", C.POINTER(C.c_int32)), ("coef", C.POINTER(C.c_int32)),
                ("sense", C.POINTER(C.c_int8)), ("rhs", C.POINTER(C.c_int64))]


class dd_options(C.Structure):
    _fields_ = [("nodes_per_lane", C.c_int32), ("waves_per_block", C.c_int32), ("ckpt_every", C.c_int32),
                ("lds_budget", C.c_int32), ("no_graphs", C.c_int32), ("adj_route_dense", C.c_int32),
                ("adj_replay", C.c_int32), ("lb_every", C.c_int32), ("max_device_bytes", C.c_int64)]


class dd_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("edges", C.c_int64), ("nodes", C.c_int64), ("arcs", C.c_int64),
                ("node_slots", C.c_int64), ("edge_slots", C.c_int64), ("tiles", C.c_int64),
                ("max_width", C.c_int32), ("max_len", C.c_int32), ("classes", C.c_int32), ("uncovered", C.c_int32),
                ("device_bytes", C.c_int64), ("coded_levels", C.c_int64), ("raw_levels", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dd_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 96), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("bytes_per_launch", C.c_double)]


_lib = None

# (name, argtypes) of every exported entry point
_VP = C.c_void_p
SIGNATURES = {
    "dd_last_error": ([], C.c_char_p),
    "dd_create": ([C.POINTER(dd_problem), C.POINTER(dd_options), _VP, C.POINTER(_VP)], C.c_int),
    "dd_destroy": ([_VP], C.c_int),
    "dd_get_stats": ([_VP, C.POINTER(dd_stats)], C.c_int),
    "dd_edge_map": ([_VP, _VP, _VP], C.c_int),
    "dd_set_params": ([_VP, _VP, _VP, _VP], C.c_int),
    "dd_seg_softmax": ([_VP, _VP, _VP, _VP], C.c_int),
    "dd_reset": ([_VP, _VP], C.c_int),
    "dd_set_state": ([_VP, _VP, _VP, _VP], C.c_int),
    "dd_get_state": ([_VP, _VP, _VP, C.c_int32, _VP], C.c_int),
    "dd_run": ([_VP, C.c_int32, _VP], C.c_int),
    "dd_run_pass": ([_VP, C.c_int32, _VP], C.c_int),
    "dd_run_trace": ([_VP, C.c_int32, C.c_int32, _VP, _VP], C.c_int),
    "dd_num_edges": ([_VP, C.POINTER(C.c_int64)], C.c_int),
    "dd_corrupt_checkpoint": ([_VP, C.c_int32], C.c_int),
    "dd_lower_bound": ([_VP, C.POINTER(C.c_double), C.POINTER(C.c_double), _VP], C.c_int),
    "dd_row_energies": ([_VP, _VP, _VP], C.c_int),
    "dd_min_marginals": ([_VP, _VP, _VP, _VP], C.c_int),
    "dd_row_nodes": ([_VP, _VP], C.c_int),
    "dd_set_costs": ([_VP, _VP, _VP], C.c_int),
    "dd_forward_unrolled": ([_VP, C.c_int32, C.c_int32, C.POINTER(C.c_double), _VP], C.c_int),
    "dd_backward": ([_VP, C.c_double, _VP, _VP, _VP, _VP], C.c_int),
    "dd_record_serial": ([_VP, C.POINTER(C.c_int64)], C.c_int),
    "dd_pass_vjp": ([_VP, C.c_int32, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP], C.c_int),
    "dd_seg_softmax_vjp": ([_VP, _VP, _VP, _VP, _VP], C.c_int),
    "dd_profile_begin": ([_VP, C.c_int32], C.c_int),
    "dd_profile_end": ([_VP, _VP, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "dd_compile_row": ([C.POINTER(dd_problem), C.c_int32, _VP, _VP, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
    "dd_forward_unrolled_from_state": ([_VP, C.c_int32, C.c_int32, C.POINTER(C.c_double), _VP], C.c_int),
    "dd_backward_state": ([_VP, C.c_double, _VP, _VP, _VP, _VP, _VP], C.c_int),
    "dd_param_transform": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP], C.c_int),
    "dd_param_transform_vjp": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP], C.c_int),
    "dd_nonparam_update": ([_VP, _VP, _VP], C.c_int),
    "dd_smoothed": ([_VP, C.c_float, C.c_int32, _VP, _VP, _VP], C.c_int),
    "dd_smoothed_noalloc": ([_VP, C.c_float, C.c_int32, _VP, _VP, _VP], C.c_int),
    "dd_argmin_assignment": ([_VP, C.c_int32, _VP, _VP], C.c_int),
    "dd_solve": ([_VP, C.c_int32, C.c_int32, C.c_double, _VP, _VP, C.POINTER(C.c_int32), _VP], C.c_int),
    "dd_gap_integral": ([_VP, _VP, C.c_int32, C.c_double, _VP, C.POINTER(C.c_double)], C.c_int),
    "dd_get_launch": ([_VP, _VP, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "dd_set_launch": ([_VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "dd_autotune": ([_VP, C.c_char_p, C.POINTER(C.c_int32), _VP], C.c_int),
    "dd_batch_create": ([C.POINTER(dd_problem), C.c_int32, C.POINTER(dd_options), _VP, C.POINTER(_VP)], C.c_int),
    "dd_batch_destroy": ([_VP], C.c_int),
    "dd_batch_instance": ([_VP], _VP),
    "dd_batch_offsets": ([_VP, _VP, _VP, _VP], C.c_int),
    "dd_batch_run": ([_VP, C.c_int32, _VP], C.c_int),
    "dd_batch_lower_bounds": ([_VP, _VP, _VP, _VP], C.c_int),
}


def lib():
    """Load libdd.so (built in-tree by paper_2205_11638_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2205_11638_amd.build` "
                              "(the solver has no non-HIP path)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code):
    if code != DD_OK:
        raise DDError(code, lib().dd_last_error().decode())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t, dtype=None, n=None):
    """Device pointer of a contiguous CUDA tensor (checked)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (cuda) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class _ProblemArgs:
    """Keeps the numpy arrays behind a dd_problem alive."""

    def __init__(self, prob):
        self.c = np.ascontiguousarray(prob.c, dtype=np.float64)
        self.row_ptr = np.ascontiguousarray(prob.row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(prob.col, dtype=np.int32)
        self.coef = np.ascontiguousarray(prob.coef, dtype=np.int32)
        self.sense = np.ascontiguousarray(prob.sense, dtype=np.int8)
        self.rhs = np.ascontiguousarray(prob.rhs, dtype=np.int64)
        self.st = dd_problem(int(prob.n), self.c.ctypes.data_as(C.POINTER(C.c_double)), int(len(self.rhs)),
                             self.row_ptr.ctypes.data_as(C.POINTER(C.c_int64)),
                             self.col.ctypes.data_as(C.POINTER(C.c_int32)),
                             self.coef.ctypes.data_as(C.POINTER(C.c_int32)),
                             self.sense.ctypes.data_as(C.POINTER(C.c_int8)),
                             self.rhs.ctypes.data_as(C.POINTER(C.c_int64)))


def gap_integral(lb, ms, d_star):
    """(g [k], g_I): the relative dual gap of a trace and its time integral (seconds)."""
    lb = np.ascontiguousarray(lb, dtype=np.float64)
    ms = np.ascontiguousarray(ms, dtype=np.float64)
    g = np.zeros(len(lb))
    gi = C.c_double()
    _check(lib().dd_gap_integral(lb.ctypes.data_as(C.c_void_p), ms.ctypes.data_as(C.c_void_p), len(lb),
                                 float(d_star), g.ctypes.data_as(C.c_void_p), C.byref(gi)))
    return g, gi.value


def compile_row(prob, row):
    """Host-only: (widths[L], arcs[nodes] as uint32 lo | hi << 16) of row `row`'s diagram."""
    L_ = lib()
    pa = _ProblemArgs(prob)
    length = int(prob.row_ptr[row + 1] - prob.row_ptr[row])
    nodes = C.c_int64()
    _check(L_.dd_compile_row(C.byref(pa.st), int(row), None, None, 0, C.byref(nodes)))
    w = np.zeros(max(length, 1), dtype=np.int32)
    arcs = np.zeros(max(nodes.value, 1), dtype=np.uint32)
    _check(L_.dd_compile_row(C.byref(pa.st), int(row), w.ctypes.data_as(C.c_void_p), arcs.ctypes.data_as(C.c_void_p),
                             int(arcs.size), C.byref(nodes)))
    return w[:length], arcs[:nodes.value]


def _options(nodes_per_lane=0, waves_per_block=0, lds_budget=0, ckpt_every=0, graphs=True, adj_route_dense=False,
             adj_replay=False, lb_every=0, max_device_bytes=0):
    return dd_options(int(nodes_per_lane), int(waves_per_block), int(ckpt_every), int(lds_budget),
                      0 if graphs else 1, 1 if adj_route_dense else 0, 1 if adj_replay else 0, int(lb_every),
                      int(max_device_bytes))


class Instance:
    """A binary program resident on the current GPU (see include/dd.h for the semantics)."""

    def __init__(self, prob, nodes_per_lane=0, waves_per_block=0, lds_budget=0, ckpt_every=0, graphs=True,
                 adj_route_dense=False, adj_replay=False, lb_every=0, max_device_bytes=0):
        import torch
        L_ = lib()
        pa = _ProblemArgs(prob)
        opt = _options(nodes_per_lane, waves_per_block, lds_budget, ckpt_every, graphs, adj_route_dense, adj_replay,
                       lb_every, max_device_bytes)
        self._lb_every = int(lb_every) if lb_every else 1
        h = C.c_void_p()
        # input validation and compilation run on the host before any HIP call
        stream = _stream() if torch.cuda.is_available() else None
        _check(L_.dd_create(C.byref(pa.st), C.byref(opt), stream, C.byref(h)))
        self._attach(L_, h, owned=True)

    def _attach(self, L_, h, owned):
        import torch
        self._h = h
        self._L = L_
        self._owned = owned
        st = dd_stats()
        _check(L_.dd_get_stats(h, C.byref(st)))
        self.stats = st.as_dict()
        self.n, self.m, self.E = int(st.n), int(st.m), int(st.edges)
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def _borrowed(cls, L_, h):
        """View of an instance owned by someone else (a batch)."""
        self = cls.__new__(cls)
        self._attach(L_, h, owned=False)
        return self

    def close(self):
        if getattr(self, "_h", None):
            if self._owned:
                self._L.dd_destroy(self._h)
            self._h = None

    __del__ = close

    def _f32(self, n):
        import torch
        return torch.empty(n, dtype=torch.float32, device=self.device)

    def edge_map(self):
        var = np.empty(self.E, dtype=np.int32)
        row = np.empty(self.E, dtype=np.int32)
        _check(self._L.dd_edge_map(self._h, var.ctypes.data_as(C.c_void_p), row.ctypes.data_as(C.c_void_p)))
        return var, row

    def set_params(self, omega, alpha):
        import torch
        _check(self._L.dd_set_params(self._h, _dptr(omega, torch.float32, self.E), _dptr(alpha, torch.float32, self.E),
                                     _stream()))

    def seg_softmax(self, alpha_hat):
        import torch
        out = self._f32(self.E)
        _check(self._L.dd_seg_softmax(self._h, _dptr(alpha_hat, torch.float32, self.E), _dptr(out), _stream()))
        return out

    def reset(self):
        _check(self._L.dd_reset(self._h, _stream()))

    def set_state(self, lam, M):
        import torch
        _check(self._L.dd_set_state(self._h, _dptr(lam, torch.float32, self.E), _dptr(M, torch.float32, self.E),
                                    _stream()))

    def get_state(self, flushed=False):
        lam, M = self._f32(self.E), self._f32(self.E)
        _check(self._L.dd_get_state(self._h, _dptr(lam), _dptr(M), int(bool(flushed)), _stream()))
        return lam, M

    def run(self, T):
        _check(self._L.dd_run(self._h, int(T), _stream()))

    def run_trace(self, T, lb_every=0):
        """T iterations with the bound after every lb_every of them, recorded on the device: float64 [T // k]."""
        import torch
        k = int(lb_every) if lb_every else getattr(self, "_lb_every", 1)
        n = int(T) // k
        out = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        _check(self._L.dd_run_trace(self._h, int(T), k, _dptr(out), _stream()))
        return out[:n]

    def num_edges(self):
        v = C.c_int64()
        _check(self._L.dd_num_edges(self._h, C.byref(v)))
        return v.value

    def corrupt_checkpoint(self, index):
        """Test hook: perturb stored checkpoint `index` so that the next backward fails (DD_E_CHECKPOINT)."""
        _check(self._L.dd_corrupt_checkpoint(self._h, int(index)))

    def run_pass(self, direction):
        _check(self._L.dd_run_pass(self._h, int(direction), _stream()))

    def lower_bound(self):
        lb, dl = C.c_double(), C.c_double()
        _check(self._L.dd_lower_bound(self._h, C.byref(lb), C.byref(dl), _stream()))
        return lb.value, dl.value

    def row_energies(self):
        out = self._f32(self.m)
        _check(self._L.dd_row_energies(self._h, _dptr(out), _stream()))
        return out

    def min_marginals(self):
        m0, m1 = self._f32(self.E), self._f32(self.E)
        _check(self._L.dd_min_marginals(self._h, _dptr(m0), _dptr(m1), _stream()))
        return m0, m1

    def row_nodes(self):
        out = np.empty(self.m, dtype=np.int64)
        _check(self._L.dd_row_nodes(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def profile_begin(self, max_launches=4096):
        _check(self._L.dd_profile_begin(self._h, int(max_launches)))

    def profile_end(self):
        """{kernel name: (launches, total_ms, algorithmic bytes per launch)} since profile_begin."""
        cap = 64
        arr = (dd_kernel_time * cap)()
        cnt = C.c_int32()
        _check(self._L.dd_profile_end(self._h, C.cast(arr, C.c_void_p), cap, C.byref(cnt)))
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms), float(arr[i].bytes_per_launch))
                for i in range(min(cnt.value, cap))}

    def set_costs(self, c):
        import torch
        _check(self._L.dd_set_costs(self._h, _dptr(c, torch.float32, self.n), _stream()))

    def forward_unrolled(self, T, ckpt_every=0):
        lb = C.c_double()
        _check(self._L.dd_forward_unrolled(self._h, int(T), int(ckpt_every), C.byref(lb), _stream()))
        return lb.value

    def backward(self, dlb=1.0):
        """(d_omega [E], d_alpha [E], d_c [n]) of dlb * LB of the recorded unrolled forward."""
        dw, da, dc = self._f32(self.E), self._f32(self.E), self._f32(self.n)
        _check(self._L.dd_backward(self._h, float(dlb), _dptr(dw), _dptr(da), _dptr(dc), _stream()))
        return dw, da, dc

    def record_serial(self):
        """Serial of the recorded unrolled forward (-1: none valid)."""
        v = C.c_int64()
        _check(self._L.dd_record_serial(self._h, C.byref(v)))
        return v.value

    def forward_unrolled_from_state(self, T, ckpt_every=0):
        lb = C.c_double()
        _check(self._L.dd_forward_unrolled_from_state(self._h, int(T), int(ckpt_every), C.byref(lb), _stream()))
        return lb.value

    def backward_state(self, dlb=1.0):
        """(d_omega, d_alpha, d_lam0, d_M0) of dlb * LB of the recorded unrolled forward ([E] each)."""
        outs = [self._f32(self.E) for _ in range(4)]
        _check(self._L.dd_backward_state(self._h, float(dlb), *[_dptr(o) for o in outs], _stream()))
        return tuple(outs)

    def param_transform(self, omega_hat, alpha_hat, theta_hat=None):
        """(omega, alpha, theta) = (sigmoid, softmax over J_i, centring over J_i) of the raw predictions."""
        import torch
        w, a = self._f32(self.E), self._f32(self.E)
        t = self._f32(self.E) if theta_hat is not None else None
        th = _dptr(theta_hat, torch.float32, self.E) if theta_hat is not None else None
        _check(self._L.dd_param_transform(self._h, _dptr(omega_hat, torch.float32, self.E),
                                          _dptr(alpha_hat, torch.float32, self.E), th, _dptr(w), _dptr(a),
                                          _dptr(t) if t is not None else None, _stream()))
        return w, a, t

    def param_transform_vjp(self, omega, alpha, d_omega, d_alpha, d_theta=None):
        import torch
        dw, da = self._f32(self.E), self._f32(self.E)
        dt = self._f32(self.E) if d_theta is not None else None
        args = [_dptr(x, torch.float32, self.E) for x in (omega, alpha, d_omega, d_alpha)]
        _check(self._L.dd_param_transform_vjp(
            self._h, *args, _dptr(d_theta, torch.float32, self.E) if d_theta is not None else None, _dptr(dw),
            _dptr(da), _dptr(dt) if dt is not None else None, _stream()))
        return dw, da, dt

    def solve(self, T, max_rounds, rel_tol=1e-6):
        """Test-time driver: (lower bounds, elapsed ms) before the first round and after each round."""
        lb = np.zeros(int(max_rounds) + 1)
        ms = np.zeros(int(max_rounds) + 1)
        r = C.c_int32()
        _check(self._L.dd_solve(self._h, int(T), int(max_rounds), float(rel_tol), lb.ctypes.data_as(C.c_void_p),
                                ms.ctypes.data_as(C.c_void_p), C.byref(r), _stream()))
        return lb[:r.value + 1], ms[:r.value + 1]

    def smoothed(self, tau, flushed=False):
        """(E_tau [m], Gibbs marginals P(x_i = 1) [E]) of the smoothed subproblems."""
        E, pm = self._f32(self.m), self._f32(self.E)
        _check(self._L.dd_smoothed(self._h, float(tau), int(bool(flushed)), _dptr(E), _dptr(pm), _stream()))
        return E, pm

    def smoothed_noalloc(self, tau, E_out, p_out, flushed=False):
        """As smoothed, into caller-allocated device tensors (E_out [m], p_out [E]), with the library's
        static per-GPU scratch: the call itself allocates nothing."""
        import torch
        _check(self._L.dd_smoothed_noalloc(self._h, float(tau), int(bool(flushed)),
                                           _dptr(E_out, torch.float32, self.m), _dptr(p_out, torch.float32, self.E),
                                           _stream()))

    def argmin_assignment(self, flushed=False):
        x = self._f32(self.E)
        _check(self._L.dd_argmin_assignment(self._h, int(bool(flushed)), _dptr(x), _stream()))
        return x

    def nonparam_update(self, theta_hat):
        import torch
        _check(self._L.dd_nonparam_update(self._h, _dptr(theta_hat, torch.float32, self.E), _stream()))

    def pass_vjp(self, direction, lam_in, M_in, dlam_out, dM_out):
        import torch
        outs = [self._f32(self.E) for _ in range(4)]
        args = [_dptr(t, torch.float32, self.E) for t in (lam_in, M_in, dlam_out, dM_out)]
        _check(self._L.dd_pass_vjp(self._h, int(direction), *args, *[_dptr(o) for o in outs], _stream()))
        return tuple(outs)  # dlam_in, dM_in, d_alpha, d_omega

    def launch_shapes(self):
        """[{P, RMAX, wpb_f, wpb_b, grid_f, grid_b}] per kernel class."""
        cnt = C.c_int32()
        _check(self._L.dd_get_launch(self._h, None, 0, C.byref(cnt)))
        out = np.zeros(6 * max(cnt.value, 1), dtype=np.int32)
        _check(self._L.dd_get_launch(self._h, out.ctypes.data_as(C.c_void_p), cnt.value, C.byref(cnt)))
        keys = ("P", "RMAX", "wpb_f", "wpb_b", "grid_f", "grid_b")
        return [dict(zip(keys, map(int, out[6 * i:6 * i + 6]))) for i in range(cnt.value)]

    def set_launch(self, c, wpb_f, wpb_b, grid_f=0, grid_b=0):
        _check(self._L.dd_set_launch(self._h, int(c), int(wpb_f), int(wpb_b), int(grid_f), int(grid_b)))

    def autotune(self, cache_path=None):
        """Time launch shapes of the pass kernels and keep the fastest; True if read from the cache."""
        hit = C.c_int32()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(self._L.dd_autotune(self._h, path, C.byref(hit), _stream()))
        return bool(hit.value)

    def seg_softmax_vjp(self, alpha, d_alpha):
        import torch
        out = self._f32(self.E)
        _check(self._L.dd_seg_softmax_vjp(self._h, _dptr(alpha, torch.float32, self.E),
                                          _dptr(d_alpha, torch.float32, self.E), _dptr(out), _stream()))
        return out


class Batch:
    """Several programs packed into one device instance (include/dd.h, dd_batch_*).

    `instance` is the packed instance: per-edge / per-variable arrays are the programs'
    canonical arrays concatenated; `var_off`, `row_off`, `edge_off` give each program's slice."""

    def __init__(self, probs, **opts):
        import torch
        L_ = lib()
        pas = [_ProblemArgs(p) for p in probs]
        k = len(pas)
        arr = (dd_problem * k)(*[pa.st for pa in pas])
        opt = _options(**opts)
        b = C.c_void_p()
        stream = _stream() if torch.cuda.is_available() else None
        _check(L_.dd_batch_create(arr, k, C.byref(opt), stream, C.byref(b)))
        self._b, self._L, self.k = b, L_, k
        self.instance = Instance._borrowed(L_, C.c_void_p(L_.dd_batch_instance(b)))
        offs = [np.zeros(k + 1, dtype=np.int64) for _ in range(3)]
        _check(L_.dd_batch_offsets(b, *[o.ctypes.data_as(C.c_void_p) for o in offs]))
        self.var_off, self.row_off, self.edge_off = offs

    def close(self):
        if getattr(self, "_b", None):
            self.instance.close()
            self._L.dd_batch_destroy(self._b)
            self._b = None

    __del__ = close

    def run(self, T):
        _check(self._L.dd_batch_run(self._b, int(T), _stream()))

    def lower_bounds(self):
        """(lbs [k], dls [k]) as numpy float64 arrays."""
        lbs = np.zeros(self.k)
        dls = np.zeros(self.k)
        _check(self._L.dd_batch_lower_bounds(self._b, lbs.ctypes.data_as(C.c_void_p), dls.ctypes.data_as(C.c_void_p),
                                             _stream()))
        return lbs, dls
