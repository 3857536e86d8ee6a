"""ctypes binding of libfctn.so (argument marshalling only).

Every function of the C ABI (include/fctn.h) is exposed under its own name;
``Plan`` wraps a plan whose workspace, inputs and outputs are torch tensors on
the GPU and whose stream is a torch stream.  All arithmetic runs in the HIP
kernels of libfctn.so; there is no fallback: if the library is missing the
first call raises.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfctn.so")

FCTN_MAX_ORDER = 8
FCTN_MAX_BONDS = 28

OK, E_INVALID, E_NOMEM, E_DEVICE, E_NUMERIC, E_UNSUPPORTED, E_CANCELLED = range(7)
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}


class FctnError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {fctn_status_str(status)} (status {status})")


class fctn_desc(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("dims", ctypes.c_int64 * FCTN_MAX_ORDER),
        ("ranks", ctypes.c_int32 * FCTN_MAX_BONDS),
        ("lambda_", ctypes.c_double * FCTN_MAX_ORDER),
        ("delta", ctypes.c_double * FCTN_MAX_ORDER),
        ("rho", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("reuse", ctypes.c_int32),
        ("order_policy", ctypes.c_int32),
        ("extrap_alpha", ctypes.c_double),
        ("extrap_beta", ctypes.c_double),
    ]


class fctn_sweep_stats(ctypes.Structure):
    _fields_ = [("rel_change", ctypes.c_double), ("f_data", ctypes.c_double),
                ("f_trace", ctypes.c_double), ("objective", ctypes.c_double),
                ("ms_stage", ctypes.c_float * 8)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n != "ms_stage"}
        d["ms_stage"] = dict(zip(STAGES, [float(v) for v in self.ms_stage]))
        return d


class fctn_stats(ctypes.Structure):
    _fields_ = [("sweeps_done", ctypes.c_int32), ("rel_change", ctypes.c_double),
                ("objective", ctypes.c_double)]


STAGES = ["pair", "gram_rhs", "reduce", "solve", "transform", "reconstruct", "x_update",
          "stats"]


class fctn_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 8), ("ms", ctypes.c_double * 8),
                ("flops", ctypes.c_double * 8), ("bytes", ctypes.c_double * 8)]

    def as_dict(self):
        return {name: {"launches": self.launches[i], "ms": self.ms[i], "flops": self.flops[i],
                       "bytes": self.bytes[i]} for i, name in enumerate(STAGES)}


class fctn_request(ctypes.Structure):
    _fields_ = [("desc", fctn_desc), ("Y_dev", ctypes.c_void_p), ("mask_dev", ctypes.c_void_p),
                ("A0_dev", ctypes.c_void_p), ("X_out_dev", ctypes.c_void_p),
                ("sweeps", ctypes.c_int32), ("tag", ctypes.c_uint64)]


class fctn_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("sweeps_done", ctypes.c_int32), ("rel_change", ctypes.c_double),
                ("objective", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(fctn_desc)
_SIGS = {
    "fctn_workspace_bytes": (ctypes.c_size_t, [_D]),
    "fctn_plan": (ctypes.c_int, [_D, _P, ctypes.c_size_t, _P,
                                 ctypes.POINTER(ctypes.POINTER(ctypes.c_double)), ctypes.c_uint64,
                                 ctypes.POINTER(_P)]),
    "fctn_set_factors": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.POINTER(ctypes.c_double))]),
    "fctn_set_observed": (ctypes.c_int, [_P, _P, _P]),
    "fctn_set_factors_dev": (ctypes.c_int, [_P, _P]),
    "fctn_set_x": (ctypes.c_int, [_P, _P]),
    "fctn_get_sweep_index": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "fctn_set_sweep_index": (ctypes.c_int, [_P, ctypes.c_int64]),
    "fctn_regrow": (ctypes.c_int, [_P, _P, _P]),
    "fctn_sweep": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(fctn_sweep_stats)]),
    "fctn_sweep_many": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.c_int32]),
    "fctn_sweep_noalloc": (ctypes.c_int, [_P, ctypes.c_int32]),
    "fctn_complete": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _P,
                                     ctypes.POINTER(fctn_stats)]),
    "fctn_get_history": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(fctn_sweep_stats)]),
    "fctn_get_x": (ctypes.c_int, [_P, _P]),
    "fctn_get_factor": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "fctn_step_gram_rhs": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "fctn_step_solve": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "fctn_step_reconstruct": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "fctn_step_x_update": (ctypes.c_int, [_P, _P, ctypes.POINTER(fctn_sweep_stats)]),
    "fctn_mode_sizes": (ctypes.c_int, [_D, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64)]),
    "fctn_profile_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "fctn_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(fctn_profile), ctypes.c_int32]),
    "fctn_destroy": (ctypes.c_int, [_P]),
    "fctn_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "fctn_server_create": (ctypes.c_int, [_P, ctypes.c_size_t, ctypes.POINTER(_P), ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]),
    "fctn_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(fctn_request)]),
    "fctn_server_step": (ctypes.c_int, [_P, ctypes.POINTER(fctn_completion), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]),
    "fctn_server_cancel": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "fctn_server_query": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "fctn_server_destroy": (ctypes.c_int, [_P]),
}


def lib():
    """Load libfctn.so (built in-tree by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, where):
    if status != OK:
        raise FctnError(status, where)


# --- thin wrappers with the C names --------------------------------------

def fctn_status_str(status):
    return lib().fctn_status_str(status).decode()


def make_desc(dims, ranks, lam=1e-2, delta=0.5, rho=0.1, precision="f32", reuse=True,
              order_policy=1, extrapolation=None):
    """extrapolation: None, or (alpha, beta) of the asymmetric extrapolation."""
    d = fctn_desc()
    N = len(dims)
    d.order = N
    for k, v in enumerate(dims):
        d.dims[k] = int(v)
    for b, r in enumerate(ranks):
        d.ranks[b] = int(r)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (N,))
    delta = np.broadcast_to(np.asarray(delta, dtype=np.float64), (N,))
    for k in range(N):
        d.lambda_[k] = float(lam[k])
        d.delta[k] = float(delta[k])
    d.rho = float(rho)
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.reuse = int(bool(reuse))
    d.order_policy = int(order_policy)
    if extrapolation is not None:
        d.extrap_alpha = float(extrapolation[0])
        d.extrap_beta = float(extrapolation[1])
    return d


def fctn_workspace_bytes(desc):
    return lib().fctn_workspace_bytes(ctypes.byref(desc))


def fctn_mode_sizes(desc, k):
    s = ctypes.c_int64()
    i = ctypes.c_int64()
    _check(lib().fctn_mode_sizes(ctypes.byref(desc), k, ctypes.byref(s), ctypes.byref(i)),
           "fctn_mode_sizes")
    return s.value, i.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """One completion problem resident on the GPU (torch-owned workspace)."""

    def __init__(self, dims, ranks, lam=1e-2, delta=0.5, rho=0.1, precision="f32", reuse=True,
                 order_policy=1, device="cuda:0", stream=None, extrapolation=None, A0=None,
                 seed=0):
        """A0: initial factors (float64 arrays with the factor shapes); None
        draws them from `seed` in the library (fctn_plan's counter-based
        generator).  set_factors may replace them afterwards."""
        import torch
        self.torch = torch
        self.dims = tuple(int(v) for v in dims)
        self.ranks = tuple(int(r) for r in ranks)
        self.precision = precision
        self.desc = make_desc(dims, ranks, lam, delta, rho, precision, reuse, order_policy,
                              extrapolation)
        self.ws_bytes = fctn_workspace_bytes(self.desc)
        if self.ws_bytes == 0:
            raise FctnError(E_UNSUPPORTED if 2 <= len(dims) <= 8 else E_INVALID, "fctn_workspace_bytes")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.elem = torch.float64 if precision == "f64" else torch.float32
        h = ctypes.c_void_p()
        a0 = None
        if A0 is not None:
            arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in A0]
            a0 = (ctypes.POINTER(ctypes.c_double) * len(arrs))(
                *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs])
        _check(lib().fctn_plan(ctypes.byref(self.desc), _ptr(self.ws), self.ws_bytes,
                               _stream_handle(self.stream), a0, ctypes.c_uint64(int(seed)),
                               ctypes.byref(h)), "fctn_plan")
        self.handle = h

    # -- inputs -------------------------------------------------------------
    def set_factors(self, factors):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in factors]
        ptrs = (ctypes.POINTER(ctypes.c_double) * len(arrs))(
            *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs])
        _check(lib().fctn_set_factors(self.handle, ptrs), "fctn_set_factors")

    def set_factors_dev(self, A_dev):
        """A_dev: float64 device tensor holding every factor back to back."""
        self._keep_A = A_dev
        self._sync_inputs()
        _check(lib().fctn_set_factors_dev(self.handle, _ptr(A_dev)), "fctn_set_factors_dev")

    def set_observed(self, Y, mask):
        Y = self._dev(Y, self.elem)
        mask = self._dev(mask, self.torch.uint8)
        self._sync_inputs()
        _check(lib().fctn_set_observed(self.handle, _ptr(Y), _ptr(mask)), "fctn_set_observed")

    def set_x(self, X):
        X = self._dev(X, self.elem)
        self._sync_inputs()
        _check(lib().fctn_set_x(self.handle, _ptr(X)), "fctn_set_x")
        self._keep = X

    def regrow_from(self, old, fills):
        """Take X, the mask and the factors of `old` (same dims and precision,
        bond ranks <= this plan's), embedding the factors at this plan's ranks;
        fills: this plan's factor shapes, float64 (list of arrays or one device
        tensor with every factor back to back), read at the new entries."""
        if isinstance(fills, (list, tuple)):
            fills = self.torch.cat([self._dev(f, self.torch.float64).reshape(-1) for f in fills])
        fills = self._dev(fills, self.torch.float64)
        self._sync_inputs()
        _check(lib().fctn_regrow(self.handle, old.handle, _ptr(fills)), "fctn_regrow")

    # -- sweeps -------------------------------------------------------------
    def sweep(self, n=1, stats=False):
        st = fctn_sweep_stats() if stats else None
        _check(lib().fctn_sweep(self.handle, int(n), ctypes.byref(st) if stats else None),
               "fctn_sweep")
        return st.as_dict() if stats else None

    def sweep_noalloc(self, n=1):
        """fctn_sweep_noalloc: the sweeps with the split-K partials in the
        library's static device array."""
        _check(lib().fctn_sweep_noalloc(self.handle, int(n)), "fctn_sweep_noalloc")

    def complete(self, max_sweeps, tol=0.0, check_every=1, X_out=None):
        st = fctn_stats()
        _check(lib().fctn_complete(self.handle, int(max_sweeps), float(tol), int(check_every),
                                   _ptr(X_out) if X_out is not None else None,
                                   ctypes.byref(st)), "fctn_complete")
        return {"sweeps_done": st.sweeps_done, "rel_change": st.rel_change,
                "objective": st.objective}

    def history(self, first, count):
        arr = (fctn_sweep_stats * count)()
        _check(lib().fctn_get_history(self.handle, int(first), int(count), arr),
               "fctn_get_history")
        return [a.as_dict() for a in arr]

    # -- outputs ------------------------------------------------------------
    def x(self):
        out = self.torch.empty(self.dims, dtype=self.elem, device=self.device)
        _check(lib().fctn_get_x(self.handle, _ptr(out)), "fctn_get_x")
        self.stream.synchronize()
        return out

    @property
    def sweep_index(self):
        t = ctypes.c_int64()
        _check(lib().fctn_get_sweep_index(self.handle, ctypes.byref(t)), "fctn_get_sweep_index")
        return t.value

    def set_sweep_index(self, t):
        _check(lib().fctn_set_sweep_index(self.handle, int(t)), "fctn_set_sweep_index")

    # -- checkpoint / resume --------------------------------------------------
    def save_state(self, path):
        """Write the run's state (X, the float64 factors, the sweep index) and
        the shape it belongs to to an .npz file (no pickled objects)."""
        arrs = {"X": self.x().cpu().numpy(), "t": np.int64(self.sweep_index),
                "dims": np.asarray(self.dims, dtype=np.int64),
                "ranks": np.asarray(self.ranks, dtype=np.int64),
                "precision": np.asarray(self.precision)}
        for k in range(len(self.dims)):
            arrs["A%d" % k] = self.factor(k).cpu().numpy()
        np.savez(path, **arrs)

    def load_state(self, path):
        """Resume a run saved by save_state on a plan with the same descriptor
        (call after set_observed, which resets X)."""
        with np.load(path, allow_pickle=False) as f:
            if tuple(f["dims"]) != self.dims or tuple(f["ranks"]) != self.ranks or \
                    str(f["precision"]) != self.precision:
                raise FctnError(E_INVALID, "load_state: the state is of another problem shape")
            self.set_factors([f["A%d" % k] for k in range(len(self.dims))])
            self.set_x(f["X"])
            self.set_sweep_index(int(f["t"]))
        self.stream.synchronize()

    def factor(self, k):
        shape = factor_shape(self.dims, self.ranks, k)
        out = self.torch.empty(shape, dtype=self.torch.float64, device=self.device)
        _check(lib().fctn_get_factor(self.handle, int(k), _ptr(out)), "fctn_get_factor")
        self.stream.synchronize()
        return out

    # -- single steps ---------------------------------------------------------
    def mode_sizes(self, k):
        return fctn_mode_sizes(self.desc, k)

    def step_gram_rhs(self, k):
        s, Ik = self.mode_sizes(k)
        G = self.torch.empty((s, s), dtype=self.torch.float64, device=self.device)
        B = self.torch.empty((Ik, s), dtype=self.torch.float64, device=self.device)
        _check(lib().fctn_step_gram_rhs(self.handle, int(k), _ptr(G), _ptr(B)),
               "fctn_step_gram_rhs")
        self.stream.synchronize()
        return G, B

    def step_solve(self, k, G, B):
        G = self._dev(G, self.torch.float64)
        B = self._dev(B, self.torch.float64)
        self._sync_inputs()
        tr = ctypes.c_double()
        _check(lib().fctn_step_solve(self.handle, int(k), _ptr(G), _ptr(B), ctypes.byref(tr)),
               "fctn_step_solve")
        return tr.value

    def step_reconstruct(self, k):
        Z = self.torch.empty(self.dims, dtype=self.elem, device=self.device)
        _check(lib().fctn_step_reconstruct(self.handle, int(k), _ptr(Z)), "fctn_step_reconstruct")
        self.stream.synchronize()
        return Z

    def step_x_update(self, Z):
        Z = self._dev(Z, self.elem)
        self._sync_inputs()
        st = fctn_sweep_stats()
        _check(lib().fctn_step_x_update(self.handle, _ptr(Z), ctypes.byref(st)),
               "fctn_step_x_update")
        return st.as_dict()

    # -- per-kernel timing ---------------------------------------------------------
    def profile_enable(self, on=True):
        _check(lib().fctn_profile_enable(self.handle, int(bool(on))), "fctn_profile_enable")

    def profile_read(self, reset=True):
        out = fctn_profile()
        _check(lib().fctn_profile_read(self.handle, ctypes.byref(out), int(bool(reset))),
               "fctn_profile_read")
        return out.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib().fctn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ----------------------------------------------------------------
    def _dev(self, a, dtype):
        torch = self.torch
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=dtype).contiguous()

    def _sync_inputs(self):
        # inputs prepared on torch's current stream must be complete before the
        # plan's stream reads them
        self.torch.cuda.current_stream(self.device).synchronize()


def factor_shape(dims, ranks, k):
    N = len(dims)
    R = [[0] * N for _ in range(N)]
    b = 0
    for i in range(N):
        for j in range(i + 1, N):
            R[i][j] = R[j][i] = ranks[b]
            b += 1
    return tuple(dims[k] if j == k else R[k][j] for j in range(N))


def sweep_many(plans, nsweeps):
    arr = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
    _check(lib().fctn_sweep_many(arr, len(plans), int(nsweeps)), "fctn_sweep_many")


class Server:
    """Continuous-batching server (fctn_server_*): a torch-owned arena as the
    memory budget, `nstreams` torch streams of default priority, at most
    `max_active` resident requests with `depth` sweeps queued each.  The
    default of 3 streams gives each its own hardware queue beside the default
    stream's (4 hardware queues per process): with 4, two streams of a fresh
    process can land on one queue and run in order (measured 159 against 210
    completions/s at saturation; 242 when the 4 land on distinct queues)."""

    def __init__(self, arena_bytes, nstreams=3, max_active=16, depth=2, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.arena_bytes = int(arena_bytes) // 256 * 256
        self.arena = torch.empty(self.arena_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        self.base = (base + 255) // 256 * 256
        self.streams = [torch.cuda.Stream(self.device) for _ in range(nstreams)]
        handles = (ctypes.c_void_p * nstreams)(*[s.cuda_stream for s in self.streams])
        h = ctypes.c_void_p()
        _check(lib().fctn_server_create(ctypes.c_void_p(self.base), self.arena_bytes, handles,
                                        nstreams, max_active, depth, ctypes.byref(h)),
               "fctn_server_create")
        self.handle = h
        self.keep = {}
        self._done = (fctn_completion * 256)()

    def submit(self, tag, dims, ranks, Y, mask, A0, sweeps, lam=1e-2, delta=0.5, rho=0.1,
               precision="bf16x3", reuse=True, order_policy=1, extrapolation=None, X_out=None):
        """Queue a request.  Y, mask: device tensors (elem, uint8); A0: float64
        device tensor with every factor back to back.  The completed X is
        returned by step() in X_out (a contiguous elem tensor of the problem's
        shape), or in a tensor allocated here if X_out is None; a caller that
        serves at a high rate passes preallocated ones, since a device allocation
        that misses torch's cache can synchronize the device."""
        torch = self.torch
        desc = make_desc(dims, ranks, lam, delta, rho, precision, reuse, order_policy,
                         extrapolation)
        elem = torch.float64 if precision == "f64" else torch.float32
        shape = tuple(int(d) for d in dims)
        if X_out is None:
            X = torch.empty(shape, dtype=elem, device=self.device)
        else:
            if tuple(X_out.shape) != shape or X_out.dtype != elem or not X_out.is_contiguous():
                raise FctnError(E_INVALID, "Server.submit: X_out of the wrong shape or type")
            X = X_out
        req = fctn_request()
        req.desc = desc
        req.Y_dev = Y.data_ptr()
        req.mask_dev = mask.data_ptr()
        req.A0_dev = A0.data_ptr()
        req.X_out_dev = X.data_ptr()
        req.sweeps = int(sweeps)
        req.tag = int(tag)
        # inputs prepared on torch's current stream must be complete before
        # the server's streams read them
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().fctn_server_submit(self.handle, ctypes.byref(req)), "fctn_server_submit")
        self.keep[int(tag)] = (Y, mask, A0, X)

    def step(self):
        """Non-blocking progress; returns a list of (completion dict, X tensor)."""
        n = ctypes.c_int32()
        _check(lib().fctn_server_step(self.handle, self._done, len(self._done), ctypes.byref(n)),
               "fctn_server_step")
        out = []
        for i in range(n.value):
            c = self._done[i].as_dict()
            out.append((c, self.keep.pop(c["tag"])[3]))
        return out

    def cancel(self, tag):
        """Cancel a queued or resident request (fctn_server_cancel); its
        completion, status E_CANCELLED, comes from a later step()."""
        _check(lib().fctn_server_cancel(self.handle, ctypes.c_uint64(int(tag))),
               "fctn_server_cancel")

    def query(self):
        q = ctypes.c_int32()
        a = ctypes.c_int32()
        u = ctypes.c_size_t()
        _check(lib().fctn_server_query(self.handle, ctypes.byref(q), ctypes.byref(a),
                                       ctypes.byref(u)), "fctn_server_query")
        return q.value, a.value, u.value

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib().fctn_server_destroy(self.handle)
            self.handle = None
